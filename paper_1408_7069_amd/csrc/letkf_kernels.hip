// gfx950 kernels of the local ETKF frame (Gray et al., arXiv:1408.7069).
//
// k_analysis: one wavefront per (instance, domain) work item, all items of a
// frame in one launch.  Per item (Sec. 4.2):
//   1. node patch of the forecast ensemble into LDS (fused form: a X_a + V,
//      Sec. 3.1.2 member prediction), member = lane;
//   2. member means, the Fried slopes of the observation region (App. B) as
//      LDS rows, scaled by sqrt(g) = f / sqrt(s r) (taper on Sigma_w^{-1/2},
//      Sec. 4.1), and the scaled innovation;
//   3. Gram Y^T Y on the matrix cores (FP32 MFMA 16x16x4; FP64 MFMA in FP64
//      mode), A~ = (m-1)/rho I + Y^T Y promoted to FP64;
//   4. FP64 Cholesky A~ = L L^T with row i of L in lane i's registers;
//   5. FP64 one-sided Jacobi on the columns of L (register resident, parallel
//      round-robin ordering, column dot products summed through an LDS
//      transpose) until the columns are orthogonal: L J = U with U^T U =
//      Lambda and A~ = (U Lambda^{-1/2}) Lambda (U Lambda^{-1/2})^T;
//   6. W = sqrt(c) U Lambda^{-3/2} U^T on the matrix cores; the mean weights
//      w = A~^{-1} b come from the Cholesky factor by two triangular solves;
//   7. owned rows: X_a = (x_b + X' w) 1^T + sqrt(rho) X' W (matrix cores),
//      written straight into the global analysis ensemble (the gather).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "letkf_types.h"

namespace letkf {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// Output row of accumulator element r in `lane` (column = lane % 16): the
// FP32 16x16x4 form gives each lane four consecutive rows, the FP64 form four
// rows four apart.
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

__device__ inline double bcast_lane(double v, int k) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
  return __hiloint2double(hi, lo);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Solve L L^T w = b with row `lane` of L in x[] and b_lane in b: forward then
// backward substitution; returns w_lane.  invd: 1 / L_kk (LDS).
__device__ inline double cholesky_solve64(const double x[64], const double *invd, double b,
                                          int lane) {
  double r = b, z = 0.0;
#pragma unroll
  for (int j = 0; j < 64; ++j) {
    const double zj = bcast_lane(r, j) * invd[j];
    if (lane == j) z = zj;
    if (lane > j) r = fma(-x[j], zj, r);
  }
  double w = 0.0;
#pragma unroll
  for (int i = 63; i >= 0; --i) {
    const double s = wave_sum(lane > i ? x[i] * w : 0.0);
    if (lane == i) w = (z - s) * invd[i];
  }
  return w;
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// C = M^T M for a K x 64 operand M (rows of stride ld) on the matrix cores:
// the 10 upper 16x16 tiles, accumulated in registers.
template <typename T>
__device__ inline void syrk_tiles(const T *M, int ld, int ksteps, typename Mfma<T>::V acc[10],
                                  int lane) {
  const int c16 = lane & 15, k4 = lane >> 4;
  int t = 0;
#pragma unroll
  for (int I = 0; I < 4; ++I)
#pragma unroll
    for (int J = I; J < 4; ++J) acc[t++] = Mfma<T>::zero();
  for (int kk = 0; kk < ksteps; ++kk) {
    const T *row = M + (4 * kk + k4) * ld;
    T a[4];
#pragma unroll
    for (int I = 0; I < 4; ++I) a[I] = row[16 * I + c16];
    t = 0;
#pragma unroll
    for (int I = 0; I < 4; ++I)
#pragma unroll
      for (int J = I; J < 4; ++J) {
        acc[t] = Mfma<T>::mac(a[I], a[J], acc[t]);
        ++t;
      }
  }
}

// Write the symmetric 64x64 result of syrk_tiles (times alpha) row-major.
template <typename T>
__device__ inline void store_sym(const typename Mfma<T>::V acc[10], T *out, int ld, T alpha,
                                 int lane) {
  const int c16 = lane & 15;
  int t = 0;
#pragma unroll
  for (int I = 0; I < 4; ++I)
#pragma unroll
    for (int J = I; J < 4; ++J) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * I + Mfma<T>::row(lane, r), j = 16 * J + c16;
        const T v = alpha * acc[t][r];
        out[i * ld + j] = v;
        if (I != J) out[j * ld + i] = v;
      }
      ++t;
    }
}

// Column sums of a 64 x 32 block held one row per lane (value k of lane i =
// f(k) in lane i): returns the sum of column (lane & 31) in lanes k and k+32.
template <typename F>
__device__ inline double colsum32(F f, double *tbuf, int lane) {
#pragma unroll
  for (int k = 0; k < 32; ++k) tbuf[lane * 33 + k] = f(k);
  __syncthreads();
  const int col = lane & 31, r0 = (lane >> 5) * 32;
  double s = 0.0;
#pragma unroll 8
  for (int r = 0; r < 32; ++r) s += tbuf[(r0 + r) * 33 + col];
  __syncthreads();
  return s + __shfl_xor(s, 32, 64);
}

// Column sums of a 64 x 64 block (value k of lane i = f(k)): lane j gets
// the sum of column j.
template <typename F>
__device__ inline double colsum64(F f, double *tbuf, int lane) {
  const double a = colsum32([&](int k) { return f(k); }, tbuf, lane);
  const double b = colsum32([&](int k) { return f(32 + k); }, tbuf, lane);
  return lane < 32 ? a : b;
}

// Cholesky of the SPD matrix whose row `lane` is x[0..63] (in place: row i
// of L, zero above the diagonal).  col: 64 doubles of LDS; invd (may be
// NULL): 64 doubles of LDS that receive 1 / L_kk.
__device__ inline void cholesky64(double x[64], double *col, double *invd, int lane) {
#pragma unroll
  for (int k = 0; k < 64; ++k) {
    const double akk = bcast_lane(x[k], k);
    const double lkk = sqrt(akk);
    if (invd && lane == 0) invd[k] = 1.0 / lkk;
    const double l = lane > k ? x[k] / lkk : 0.0;
    x[k] = lane > k ? l : (lane == k ? lkk : 0.0);
    col[lane] = l;
    __syncthreads();
#pragma unroll
    for (int j = k + 1; j < 64; ++j) x[j] = fma(-l, col[j], x[j]);
    __syncthreads();
  }
}

// One-sided Jacobi on the columns of x (row = lane) in the round-robin order:
// positions (k, 63 - k), k < 32, are rotated together; then positions 1..63
// shift by one (position 0 fixed), so 63 rounds visit every pair once and
// return every column to its place.  Rotations zero the column inner product
// (t = sign(z) / (|z| + sqrt(1 + z^2)), z = (|x_q|^2 - |x_p|^2) / (2 x_p.x_q)).
// Stops after the first sweep whose largest |x_p.x_q| / (|x_p| |x_q|) <= tol.
// Returns the number of sweeps, or -sweeps when it did not converge.
__device__ inline int jacobi64(double x[64], double *tbuf, double *rot, double tol,
                               int max_sweeps, int lane) {
  double nrm = colsum64([&](int k) { return x[k] * x[k]; }, tbuf, lane);
  int sweep = 0;
  bool done = false;
  while (!done && sweep < max_sweeps) {
    double maxoff = 0.0;
    for (int round = 0; round < 63; ++round) {
      const double gam = colsum32([&](int k) { return x[k] * x[63 - k]; }, tbuf, lane);
      const double alp = nrm;
      const double bet = __shfl(nrm, 63 - lane, 64);
      double cs = 1.0, sn = 0.0, t = 0.0;
      if (lane < 32 && gam != 0.0) {
        maxoff = fmax(maxoff, fabs(gam) / sqrt(alp * bet));
        const double zeta = (bet - alp) / (2.0 * gam);
        t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        cs = 1.0 / sqrt(1.0 + t * t);
        sn = cs * t;
      }
      if (lane < 32) {
        rot[2 * lane] = cs;
        rot[2 * lane + 1] = sn;
      }
      const double nal = alp - t * gam;
      const double nbe = bet + t * gam;
      const double nbe_mirror = __shfl(nbe, 63 - lane, 64);
      const double nrm_new = lane < 32 ? nal : nbe_mirror;
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 32; ++k) {
        const double c_ = rot[2 * k], s_ = rot[2 * k + 1];
        const double xp = x[k], xq = x[63 - k];
        x[k] = c_ * xp - s_ * xq;
        x[63 - k] = s_ * xp + c_ * xq;
      }
      const double last = x[63];
#pragma unroll
      for (int j = 63; j >= 2; --j) x[j] = x[j - 1];
      x[1] = last;
      const int src = lane == 0 ? 0 : (lane == 1 ? 63 : lane - 1);
      nrm = __shfl(nrm_new, src, 64);
      __syncthreads();
    }
    ++sweep;
    done = wave_max(maxoff) <= tol;
  }
  return done ? sweep : -sweep;
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
  int32_t *flags;
  const uint32_t *frame;  // frame counter of the bank draws (device)
  double jtol;
  int32_t max_sweeps;
  int32_t off_xs, off_xm, off_sg, off_dd, off_yb, off_pn, off_s, off_u;
};

__device__ inline int xcd_item(int b, int grid) {
  // blocks are dealt to the 8 XCDs round-robin; give XCD x the contiguous run
  // of items [x * per, (x + 1) * per).  grid is a multiple of 8.
  const int per = grid >> 3;
  return (b & 7) * per + (b >> 3);
}

template <typename T, bool FUSED>
__global__ __launch_bounds__(64) void k_analysis(const AnaArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x;
  int item = A.xcd_order ? xcd_item((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
  item += A.item_base;
  if (item >= A.n_items) return;
  const DomItem it = A.items[item];
  const InstDesc in = A.inst[it.inst];
  const int m = in.m;
  const int np = it.n_patch, nown = it.n_own, nobs = it.n_obs;
  const int p = 2 * nobs, p4 = (p + 3) & ~3;

  T *xs = (T *)(smem + A.off_xs);
  T *xm = (T *)(smem + A.off_xm);
  double *sg = (double *)(smem + A.off_sg);
  double *dd = (double *)(smem + A.off_dd);
  T *yb = (T *)(smem + A.off_yb);
  int *pn = (int *)(smem + A.off_pn);
  double *sm = (double *)(smem + A.off_s);  // 6 x 64 doubles of small scratch
  unsigned char *U = smem + A.off_u;

  // ---- 1. node patch of X_b ----
  const int my_node = lane < np ? A.patch_node[it.patch_off + lane] : 0;
  pn[lane] = my_node;
  BankDraw bd{};
  const bool use_bank = FUSED && A.noise_bank;
  if (use_bank && lane < m) bd = bank_draw(in, *A.frame, lane);
  const T a = (T)in.a;
  for (int r = 0; r < np; ++r) {
    const int g = __builtin_amdgcn_readlane(my_node, r);
    T v = (T)0;
    if (lane < m) {
      const int64_t e = in.x_off + (int64_t)g * m + lane;
      const T x = A.x_in[e];
      if (FUSED) {
        T noise;
        if (use_bank) {
          const int gi = A.node_ij[2 * (in.node_off + g)], gj = A.node_ij[2 * (in.node_off + g) + 1];
          noise = (T)bank_value(A.bank, bd, gi, gj);
        } else {
          noise = A.v_in[e];
        }
        v = fma_t(a, x, noise);
      } else {
        v = x;
      }
    }
    xs[r * kXsStride + lane] = v;
  }
  __syncthreads();
  if (lane < np) {
    T s = (T)0;
    for (int j = 0; j < m; ++j) s += xs[lane * kXsStride + j];
    xm[lane] = s / (T)m;
  }
  __syncthreads();

  // ---- 2. local slopes, weights and innovation ----
  uint32_t my_corner = 0;
  int bad = 0;
  if (lane < nobs) {
    my_corner = A.obs_corner[it.obs_off + lane];
    const int k = A.obs_sub[it.obs_off + lane];
    const int ca = my_corner & 255, cb = (my_corner >> 8) & 255, cc = (my_corner >> 16) & 255,
              cd = my_corner >> 24;
    const T ybx = (T)0.5 * ((xm[cb] - xm[ca]) + (xm[cd] - xm[cc]));
    const T yby = (T)0.5 * ((xm[cc] - xm[ca]) + (xm[cd] - xm[cb]));
    const double f = in.taper_c > 0.0 ? gaspari_cohn(A.obs_dist[it.obs_off + lane] / in.taper_c) : 1.0;
    const double rx = A.r_diag[in.y_off + k], ry = A.r_diag[in.y_off + in.n_subaps + k];
    const double sgx = f / sqrt(in.r_scale * rx), sgy = f / sqrt(in.r_scale * ry);
    const double yx = (double)A.y[in.y_off + k], yy = (double)A.y[in.y_off + in.n_subaps + k];
    bad = !(isfinite(yx) && isfinite(yy));
    sg[lane] = sgx;
    sg[nobs + lane] = sgy;
    dd[lane] = sgx * (yx - (double)ybx);
    dd[nobs + lane] = sgy * (yy - (double)yby);
    yb[lane] = ybx;
    yb[nobs + lane] = yby;
  }
  bad = __any(bad);
  __syncthreads();
  T *ys = (T *)U;  // [p4][kYsStride], K-major MFMA operand
  for (int q = 0; q < nobs; ++q) {
    const uint32_t cw = (uint32_t)__builtin_amdgcn_readlane((int)my_corner, q);
    const int ca = cw & 255, cb = (cw >> 8) & 255, cc = (cw >> 16) & 255, cd = cw >> 24;
    const T pa = xs[ca * kXsStride + lane], pb = xs[cb * kXsStride + lane];
    const T pc = xs[cc * kXsStride + lane], pd = xs[cd * kXsStride + lane];
    const T sx = (T)0.5 * ((pb - pa) + (pd - pc)) - yb[q];
    const T sy = (T)0.5 * ((pc - pa) + (pd - pb)) - yb[nobs + q];
    ys[q * kYsStride + lane] = lane < m ? (T)sg[q] * sx : (T)0;
    ys[(nobs + q) * kYsStride + lane] = lane < m ? (T)sg[nobs + q] * sy : (T)0;
  }
  for (int q = p; q < p4; ++q) ys[q * kYsStride + lane] = (T)0;
  __syncthreads();
  double bj = 0.0;  // b = Y^T sqrt(g) d, member = lane
  for (int s = 0; s < p; ++s) bj = fma((double)ys[s * kYsStride + lane], dd[s], bj);

  // ---- 3. Gram on the matrix cores ----
  typename Mfma<T>::V acc[10];
  syrk_tiles<T>(ys, kYsStride, p4 / 4, acc, lane);
  __syncthreads();
  T *gram = (T *)U;  // [64][kXsStride]
  store_sym<T>(acc, gram, kXsStride, (T)1, lane);
  __syncthreads();
  const double c = (double)(m - 1) / in.rho;
  double x[64];
#pragma unroll
  for (int k = 0; k < 64; ++k) x[k] = (double)gram[lane * kXsStride + k] + (k == lane ? c : 0.0);
  __syncthreads();

  // ---- 4./5. FP64 Cholesky and one-sided Jacobi ----
  double *tbuf = (double *)U;             // 64 x 33 doubles
  double *rot = sm;                       // 64 doubles
  double *col = sm + 64;                  // 64 doubles
  double *invd = sm + 192;                // 1 / L_kk
  cholesky64(x, col, invd, lane);
  __syncthreads();
  // w = A~^{-1} b from the factor itself, independent of the Jacobi stop
  const double wbar = cholesky_solve64(x, invd, bj, lane);
  const int sweeps = jacobi64(x, tbuf, rot, A.jtol, A.max_sweeps, lane);
  const bool conv = sweeps > 0;

  // ---- 6. transform: lambda, W = sqrt(c) U Lambda^{-3/2} U^T, w ----
  const double lam = colsum64([&](int k) { return x[k] * x[k]; }, tbuf, lane);  // lane j: eigenvalue j
  double *lamv = sm + 128;                      // lambda^{-3/4}
  double *wv = sm + 256;                        // w
  double *xa_mean = sm + 320;                   // analysis mean of the owned rows
  lamv[lane] = 1.0 / sqrt(lam * sqrt(lam));
  __syncthreads();
  T *ut = (T *)U;     // [64][kYsStride]: (U Lambda^{-3/4})^T, K-major (tbuf is dead)
#pragma unroll
  for (int k = 0; k < 64; ++k) ut[k * kYsStride + lane] = (T)(x[k] * lamv[k]);
  wv[lane] = wbar;
  __syncthreads();
  syrk_tiles<T>(ut, kYsStride, 16, acc, lane);
  __syncthreads();
  T *wmat = ut;      // W row-major [64][kYsStride]
  store_sym<T>(acc, wmat, kYsStride, (T)sqrt(c), lane);
  __syncthreads();

  // ---- 7. owned rows: X_a = (x_b + X' w) 1^T + sqrt(rho) X' W ----
  const bool keep_forecast = bad || !conv || !isfinite(lam);
  if (lane == 0) A.flags[item] = (bad || !isfinite(lam) ? 1 : 0) | (conv ? 0 : 2);
  if (lane < nown) {
    double s = (double)xm[lane];
    const double mu = (double)xm[lane];
    for (int k = 0; k < m; ++k) s = fma((double)xs[lane * kXsStride + k] - mu, wv[k], s);
    xa_mean[lane] = s;
  }
  __syncthreads();
  const T srho = (T)sqrt(in.rho);
  const int c16 = lane & 15, k4 = lane >> 4;
  for (int I = 0; I * 16 < nown; ++I) {
    typename Mfma<T>::V o[4];
#pragma unroll
    for (int J = 0; J < 4; ++J) o[J] = Mfma<T>::zero();
    const int ia = 16 * I + c16;
    const T mu = ia < nown ? xm[ia] : (T)0;
    for (int kk = 0; kk < 16; ++kk) {
      const int k = 4 * kk + k4;
      const T av = (ia < nown && k < m) ? xs[ia * kXsStride + k] - mu : (T)0;
#pragma unroll
      for (int J = 0; J < 4; ++J) o[J] = Mfma<T>::mac(av, wmat[k * kYsStride + 16 * J + c16], o[J]);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * I + Mfma<T>::row(lane, r);
      if (i < nown) {
        const int g = pn[i];
        const T base = (T)xa_mean[i];
#pragma unroll
        for (int J = 0; J < 4; ++J) {
          const int j = 16 * J + c16;
          if (j < m) {
            const T v = keep_forecast ? xs[i * kXsStride + j] : base + srho * o[J][r];
            A.x_out[in.x_off + (int64_t)g * m + j] = v;
          }
        }
      }
    }
  }
}

// Forecast X_b = a X_a + V over every instance (blockIdx.y = instance).
template <typename T>
__global__ void k_forecast(const InstDesc *insts, const int32_t *node_ij, const T *xa, const T *v,
                           const float *bank, const uint32_t *frame, T *xb) {
  const InstDesc in = insts[blockIdx.y];
  const int64_t n = (int64_t)in.n_nodes * in.m;
  const T a = (T)in.a;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    T noise;
    if (v) {
      noise = v[in.x_off + e];
    } else {
      const int member = (int)(e % in.m);
      const int node = (int)(e / in.m);
      const BankDraw bd = bank_draw(in, *frame, member);
      noise = (T)bank_value(bank, bd, node_ij[2 * (in.node_off + node)],
                            node_ij[2 * (in.node_off + node) + 1]);
    }
    xb[in.x_off + e] = fma_t(a, xa[in.x_off + e], noise);
  }
}

__global__ void k_frame_advance(uint32_t *frame) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *frame += 1u;
}

// Fried slopes of one phase vector per instance (blockIdx.y = instance).
template <typename T>
__global__ void k_slopes(const InstDesc *insts, const int32_t *subap_nodes, const T *phase,
                         T *slopes) {
  const InstDesc in = insts[blockIdx.y];
  const int64_t node0 = in.node_off;  // phase offset (nodes) of this instance
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < in.n_subaps; k += gridDim.x * blockDim.x) {
    const int32_t *c = subap_nodes + 4 * (in.y_off / 2 + k);
    const T pa = phase[node0 + c[0]], pb = phase[node0 + c[1]];
    const T pc = phase[node0 + c[2]], pd = phase[node0 + c[3]];
    slopes[in.y_off + k] = (T)0.5 * ((pb - pa) + (pd - pc));
    slopes[in.y_off + in.n_subaps + k] = (T)0.5 * ((pc - pa) + (pd - pb));
  }
}

// Member mean per node (blockIdx.y = instance).
template <typename T>
__global__ void k_mean(const InstDesc *insts, const T *x, T *mean) {
  const InstDesc in = insts[blockIdx.y];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < in.n_nodes; i += gridDim.x * blockDim.x) {
    T s = (T)0;
    for (int j = 0; j < in.m; ++j) s += x[in.x_off + (int64_t)i * in.m + j];
    mean[in.node_off + i] = s / (T)in.m;
  }
}

// Stand-alone SPD eigensolve, one wavefront per matrix.
__global__ __launch_bounds__(64) void k_eigh_spd(const double *Am, int m, double tol, int max_sweeps,
                                                 double *Q, double *lam_out, int32_t *sweeps_out) {
  __shared__ double tbuf[64 * 33 + 128];
  const int lane = threadIdx.x;
  const double *Ab = Am + (int64_t)blockIdx.x * m * m;
  double x[64];
#pragma unroll
  for (int k = 0; k < 64; ++k) {
    double v;
    if (lane < m && k < m) v = Ab[lane * m + k];
    else v = (k == lane) ? 1.0 : 0.0;
    x[k] = v;
  }
  double *rot = tbuf + 64 * 33;
  double *col = rot + 64;
  cholesky64(x, col, nullptr, lane);
  const int sw = jacobi64(x, tbuf, rot, tol, max_sweeps, lane);
  const double lam = colsum64([&](int k) { return x[k] * x[k]; }, tbuf, lane);
  col[lane] = 1.0 / sqrt(lam);
  __syncthreads();
  if (lane < m) {
    double *Qb = Q + (int64_t)blockIdx.x * m * m;
#pragma unroll
    for (int k = 0; k < 64; ++k)
      if (k < m) Qb[lane * m + k] = x[k] * col[k];
    lam_out[(int64_t)blockIdx.x * m + lane] = lam;
  }
  if (lane == 0 && sweeps_out) sweeps_out[blockIdx.x] = sw;
}

}  // namespace letkf

// ---------------------------------------------------------------------------
// Launch wrappers called by the host side.
using namespace letkf;

extern "C" hipError_t letkf_launch_analysis_f32(const void *args, int fused, int grid,
                                                size_t lds, hipStream_t s) {
  const AnaArgs<float> &A = *(const AnaArgs<float> *)args;
  if (fused)
    hipLaunchKernelGGL((k_analysis<float, true>), dim3(grid), dim3(64), lds, s, A);
  else
    hipLaunchKernelGGL((k_analysis<float, false>), dim3(grid), dim3(64), lds, s, A);
  return hipGetLastError();
}

extern "C" hipError_t letkf_launch_analysis_f64(const void *args, int fused, int grid,
                                                size_t lds, hipStream_t s) {
  const AnaArgs<double> &A = *(const AnaArgs<double> *)args;
  if (fused)
    hipLaunchKernelGGL((k_analysis<double, true>), dim3(grid), dim3(64), lds, s, A);
  else
    hipLaunchKernelGGL((k_analysis<double, false>), dim3(grid), dim3(64), lds, s, A);
  return hipGetLastError();
}

extern "C" const void *letkf_analysis_kernel(int fp64, int fused) {
  if (fp64) return fused ? (const void *)k_analysis<double, true> : (const void *)k_analysis<double, false>;
  return fused ? (const void *)k_analysis<float, true> : (const void *)k_analysis<float, false>;
}

extern "C" hipError_t letkf_launch_forecast(int fp64, const InstDesc *insts, int n_inst,
                                            const int32_t *node_ij, const void *xa, const void *v,
                                            const float *bank, const uint32_t *frame, void *xb,
                                            int64_t max_elems, hipStream_t s) {
  int gx = (int)((max_elems + 255) / 256);
  if (gx > 4096) gx = 4096;
  if (gx < 1) gx = 1;
  if (fp64)
    hipLaunchKernelGGL(k_forecast<double>, dim3(gx, n_inst), dim3(256), 0, s, insts, node_ij,
                       (const double *)xa, (const double *)v, bank, frame, (double *)xb);
  else
    hipLaunchKernelGGL(k_forecast<float>, dim3(gx, n_inst), dim3(256), 0, s, insts, node_ij,
                       (const float *)xa, (const float *)v, bank, frame, (float *)xb);
  return hipGetLastError();
}

extern "C" const void *letkf_frame_advance_kernel(void) { return (const void *)k_frame_advance; }

extern "C" hipError_t letkf_launch_frame_advance(uint32_t *frame, hipStream_t s) {
  hipLaunchKernelGGL(k_frame_advance, dim3(1), dim3(64), 0, s, frame);
  return hipGetLastError();
}

extern "C" hipError_t letkf_launch_slopes(int fp64, const InstDesc *insts, int n_inst,
                                          const int32_t *subap_nodes, const void *phase,
                                          void *slopes, int max_subaps, hipStream_t s) {
  int gx = (max_subaps + 255) / 256;
  if (gx < 1) gx = 1;
  if (fp64)
    hipLaunchKernelGGL(k_slopes<double>, dim3(gx, n_inst), dim3(256), 0, s, insts, subap_nodes,
                       (const double *)phase, (double *)slopes);
  else
    hipLaunchKernelGGL(k_slopes<float>, dim3(gx, n_inst), dim3(256), 0, s, insts, subap_nodes,
                       (const float *)phase, (float *)slopes);
  return hipGetLastError();
}

extern "C" hipError_t letkf_launch_mean(int fp64, const InstDesc *insts, int n_inst, const void *x,
                                        void *mean, int max_nodes, hipStream_t s) {
  int gx = (max_nodes + 255) / 256;
  if (gx < 1) gx = 1;
  if (fp64)
    hipLaunchKernelGGL(k_mean<double>, dim3(gx, n_inst), dim3(256), 0, s, insts,
                       (const double *)x, (double *)mean);
  else
    hipLaunchKernelGGL(k_mean<float>, dim3(gx, n_inst), dim3(256), 0, s, insts, (const float *)x,
                       (float *)mean);
  return hipGetLastError();
}

extern "C" hipError_t letkf_launch_eigh(const double *A, int m, int batch, double tol, int max_sweeps,
                                        double *Q, double *lam, int32_t *sweeps, hipStream_t s) {
  hipLaunchKernelGGL(k_eigh_spd, dim3(batch), dim3(64), 0, s, A, m, tol, max_sweeps, Q, lam, sweeps);
  return hipGetLastError();
}

extern "C" size_t letkf_args_size(int fp64) {
  return fp64 ? sizeof(AnaArgs<double>) : sizeof(AnaArgs<float>);
}
