// Device-side pieces shared by the analysis kernels of the local ETKF frame
// (the 64-member workgroup layout and the wide-shape one): MFMA accumulator
// conventions, the Philox bank draws, the Gaspari-Cohn taper, the argument
// block of an analysis launch.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "letkf_types.h"

namespace letkf {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Output row of accumulator element r in `lane` (column = lane % 16): the
// FP32 16x16x4 form gives each lane four consecutive rows, the FP64 form four
// rows four apart.
template <typename T> struct Mfma;
template <> struct Mfma<float> {
  typedef f32x4 V;
  __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
  __device__ static V zero() { return V{0.f, 0.f, 0.f, 0.f}; }
  __device__ static V mac(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<double> {
  typedef f64x4 V;
  __device__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
  __device__ static V zero() { return V{0.0, 0.0, 0.0, 0.0}; }
  __device__ static V mac(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

__device__ inline float fma_t(float a, float b, float c) { return fmaf(a, b, c); }
__device__ inline double fma_t(double a, double b, double c) { return fma(a, b, c); }

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32 -> 64-bit
// products, key bumped by the Weyl constants between rounds.
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// Bank draw of one member at one frame: screen, shift and orientation.
struct BankDraw {
  int64_t base;
  int oy, ox, orient, side;
};

__device__ inline BankDraw bank_draw(const InstDesc &in, uint32_t frame, int member) {
  uint32_t c[4] = {frame, (uint32_t)member, in.instance, 0u};
  philox4x32_10(c, in.seed_lo, in.seed_hi);
  BankDraw d;
  const int side = in.bank_side;
  d.side = side;
  d.base = in.bank_off + (int64_t)(c[0] % (uint32_t)in.bank_screens) * side * side;
  d.oy = (int)(c[1] & (uint32_t)(side - 1));
  d.ox = (int)(c[2] & (uint32_t)(side - 1));
  d.orient = (int)(c[3] & 7u);
  return d;
}

__device__ inline float bank_value(const float *bank, const BankDraw &d, int i, int j) {
  int u = (d.orient & 1) ? j : i;
  int v = (d.orient & 1) ? i : j;
  if (d.orient & 2) u = -u;
  if (d.orient & 4) v = -v;
  const int mask = d.side - 1;
  return bank[d.base + (int64_t)((d.oy + u) & mask) * d.side + ((d.ox + v) & mask)];
}

// Gaspari & Cohn (1999) fifth-order compactly supported correlation of z = r/c.
__device__ inline double gaspari_cohn(double z) {
  z = fabs(z);
  if (z >= 2.0) return 0.0;
  if (z <= 1.0) return (((-0.25 * z + 0.5) * z + 0.625) * z - 5.0 / 3.0) * z * z + 1.0;
  return ((((z / 12.0 - 0.5) * z + 0.625) * z + 5.0 / 3.0) * z - 5.0) * z + 4.0 - 2.0 / (3.0 * z);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T> struct AnaArgs {
  const InstDesc *inst;
  const DomItem *items;
  int32_t item_base, n_items, xcd_order, noise_bank;  // noise_bank: V from the bank
  const int32_t *patch_node;
  const uint32_t *obs_corner;
  const int32_t *obs_sub;
  const double *obs_dist;
  const int32_t *node_ij;
  const double *r_diag;
  const T *x_in;       // X_b (split form) or the previous X_a (fused form)
  const T *v_in;       // explicit V (fused form), else NULL
  const float *bank;
  const T *y;
  T *x_out;
  T *x_mean;           // analysis mean of every node (NULL: not written)
  int32_t *flags;
  const uint32_t *frame;  // frame counter of the bank draws (device)
  const T *u_prev2;       // closed loop: the command u_{k-2} per node (NULL: none)
  const T *x_prev;        // AR(2): the analysis ensemble of the frame before x_in (NULL: none)
  T *stage;               // blend: analysed patch rows [patch entry][64] (NULL: no blend instance)
  double *stage_mean;     // blend: their member means [patch entry]
  double jtol;
  int32_t max_sweeps;
  int32_t off_xs, off_xm, off_sg, off_dd, off_yb, off_pn, off_s, off_u, off_ys;
  int32_t off_clb, off_clr;  // covariance localisation: B and the solve's columns
  int32_t round_items;        // work items of one dispatch round per XCD (CUs per XCD)
  int32_t p32;                // wide analysis, FP32 state: P updates in FP32 past the switch (NSP_MIXED)
  const int32_t *order;       // grid slot -> work item (-1: none), or NULL for the fixed orders
};

__device__ inline int xcd_item(int b, int grid) {
  // blocks are dealt to the 8 XCDs round-robin; give XCD x the contiguous run
  // of items [x * per, (x + 1) * per).  grid is a multiple of 8.
  const int per = grid >> 3;
  return (b & 7) * per + (b >> 3);
}

}  // namespace letkf
