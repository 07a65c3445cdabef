// gfx950 kernels of the local ETKF frame (Gray et al., arXiv:1408.7069).
//
// k_analysis: one 256-thread workgroup (4 wavefronts) per (instance, domain)
// work item, all items of a frame in one launch.  Per item (Sec. 4.2):
//   1. node patch of the forecast ensemble into LDS (fused form: a X_a + V,
//      Sec. 3.1.2 member prediction), member = lane;
//   2. member means, the Fried slopes of the observation region (App. B) as
//      LDS rows, scaled by sqrt(g) = f / sqrt(s r) (taper on Sigma_w^{-1/2},
//      Sec. 4.1), and the scaled innovation;
//   3. Gram Y^T Y on the matrix cores (FP32 MFMA 16x16x4; FP64 MFMA in FP64
//      mode), A~ = (m-1)/rho I + Y^T Y promoted to FP64;
//   4.-6. the transform, one of
//      NS64 (default): A~^{-1/2} by the scaled coupled Newton-Schulz
//        iteration on the FP64 matrix cores (64 x 64 products; each wave holds
//        one 16-column block of the iterates in accumulator tiles), then
//        w = A~^{-1} b = Z (Z b) / s and W = sqrt(c / s) Z;
//      NS32: the same iteration with FP32 iterates on the FP32 matrix cores,
//        w refined once in FP64;
//      EVD: FP64 Cholesky A~ = L L^T, w by two triangular solves, the FP64
//        one-sided Jacobi on the columns of L until they are orthogonal
//        (L J = U, U^T U = Lambda, A~ = (U Lambda^{-1/2}) Lambda
//        (U Lambda^{-1/2})^T), W = sqrt(c) U Lambda^{-3/2} U^T;
//   7. owned rows: X_a = (x_b + X' w) 1^T + sqrt(rho) X' W (matrix cores),
//      written straight into the global analysis ensemble (the gather).
//
// Layout of the 64 x 64 FP64 factor during the Jacobi: lane = row; the 64
// columns form 8 blocks of 8, wave q holding block q and block 7 - q in
// registers.  A Jacobi sweep pairs the columns inside each held block (7
// rounds of a round robin on 8), then runs 7 block-rounds of 8 rounds that
// pair every column of one held block with every column of the other, moving
// the blocks between waves through LDS after each block-round (block slot 0
// fixed, slots 1..7 rotating): every pair of columns meets once per sweep and
// only the block moves need a workgroup barrier.
//
// k_adjoint recomputes stages 1-6 (EVD transform) and then runs the reverse
// of stage 7 and of the transform (see the comment above it); k_adjoint_nodes
// sums the per-domain slope adjoints per slope, applies D^T and hands the
// adjoint of the previous analysis ensemble back.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>
#include <type_traits>

#include "letkf_device.h"
#include "letkf_types.h"

namespace letkf {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;


__device__ inline double bcast_lane(double v, int k) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
  return __hiloint2double(hi, lo);
}


// LDS traffic of one wavefront only: in-order within the wave, so a compiler
// barrier suffices between the writes and the reads of other lanes.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 1/sqrt(x) from the hardware estimate refined by Newton steps.
__device__ inline double rsq_nr(double x, int steps) {
  double y = __builtin_amdgcn_rsq(x);
  for (int i = 0; i < steps; ++i) y = y * fma(-0.5 * x * y, y, 1.5);
  return y;
}

// ------------------------------------------------------------ LDS scratch
// Small FP64 scratch (offsets in doubles).  The forward analysis uses the
// first kFwdScratch; the Jacobi paths (adjoint, batched eigensolver) all.
// the patch-node area (ints): patch nodes [0, 64), their packed (i, j)
// [64, 128), the corner words of the observation subapertures [128, 192),
// then u_{k-2} at the patch nodes (64 elements of the state type)
constexpr int kPnCw = 128, kPnU = 192;
constexpr int S_VEC = 0;       // 64: b = Yt^T sqrt(g) d (residual / z of the solves)
constexpr int S_WV = 64;       // 64: w
constexpr int S_XAM = 128;     // 64: analysis mean of the owned rows
constexpr int S_COL = 192;     // 2 x 64: Z b of the mean weights
constexpr int S_RES = 320;     // 4 waves: partial sums of squares (norm, residual)
constexpr int kFwdScratch = 328;
constexpr int S_INVD = 328;    // 64: 1 / L_kk
constexpr int S_LAM = 392;     // 64: lambda^{-3/4}
constexpr int S_NRM = 456;     // 4 waves x 16: column norms by register slot
constexpr int S_MAX = 520;     // 2 x 4 waves: last round above tol, by block-move parity
constexpr int S_XN = 528;      // 4 waves x 16: norms in flight between waves
constexpr int S_LAMV = 592;    // 64: lambda
constexpr int S_TOTAL = 656;
constexpr int kXchBytes = kWaves * 8 * 64 * 8;   // one block of every wave in flight

// The 64 columns form 8 blocks of 8; wave q holds block q in X[0..7] and
// block 7 - q in Y[0..7] (ascending columns), lane = row.
__device__ inline int pos_x(int q, int j) { return 8 * q + j; }
__device__ inline int pos_y(int q, int j) { return 56 - 8 * q + j; }

// Lane permutation within 16-lane rows (every source lane valid).
template <int CTRL> __device__ inline double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// Sum over the 8 lanes of each aligned group of 8 (quad swaps, then the two
// quads of each half-row), result in all 8 lanes.
__device__ inline double sum8_dpp(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  return v;
}

// a + b after swapping the upper half-wave of a with the lower half of b
// (v_permlane32_swap): lanes 0..31 get a_l + a_{l+32}, lanes 32..63 get
// b_{l-32} + b_l.
__device__ inline double swap_sum32(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(a),
                                                   (unsigned)__double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(a),
                                                   (unsigned)__double2hiint(b), false, false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}

// The same between neighbouring 16-lane rows (v_permlane16_swap): rows 0 and
// 2 get a_l + a_{l+16}, rows 1 and 3 get b_{l-16} + b_l.
__device__ inline double swap_sum16(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(a),
                                                   (unsigned)__double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(a),
                                                   (unsigned)__double2hiint(b), false, false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}

// Sum over the 64 lanes in registers (DPP within 16-lane rows, then the
// row swaps), result in every lane.
__device__ inline double wave_sum_dpp(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  v = swap_sum16(v, v);
  return swap_sum32(v, v);
}

// Sum over the four 16-lane rows (lanes l, l + 16, l + 32, l + 48), in every lane.
__device__ inline double rows_sum(double v) {
  v = swap_sum16(v, v);
  return swap_sum32(v, v);
}

// Sums over the 64 rows (lanes) of 8 per-lane values f(j) of this wave:
// returns the sum of value (lane >> 3) in the 8 lanes of each group.  A
// reduce-scatter in registers: lane bit 5 keeps j or j + 4, bit 4 one of the
// remaining pairs, bit 3 (lane ^ 8 by DPP row_ror:8) the last one, then the
// sum over the group of 8 lanes.
template <typename F> __device__ inline double group_sums8(F f, int r) {
  double v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = f(j);
  const double w0 = swap_sum32(v[0], v[4]), w1 = swap_sum32(v[1], v[5]);
  const double w2 = swap_sum32(v[2], v[6]), w3 = swap_sum32(v[3], v[7]);
  const double u0 = swap_sum16(w0, w2), u1 = swap_sum16(w1, w3);
  const bool odd = (r & 8) != 0;
  const double send = odd ? u0 : u1, keep = odd ? u1 : u0;
  return sum8_dpp(keep + dpp_f64<0x128>(send));
}

// Column sums of the distributed 64 x 64 block (f applied to each element)
// written to out[column].
template <typename F>
__device__ inline void column_sums(const double X[8], const double Y[8], F f, double *out, int q,
                                   int r) {
  const double a = group_sums8([&](int j) { return f(X[j]); }, r);
  if ((r & 7) == 0) out[pos_x(q, r >> 3)] = a;
  const double b = group_sums8([&](int j) { return f(Y[j]); }, r);
  if ((r & 7) == 0) out[pos_y(q, r >> 3)] = b;
}

constexpr int kLaStride = 65;  // FP64 64 x 64 matrix in LDS (row stride)

// Right-looking blocked Cholesky A = L L^T of the SPD matrix in LDS (row-major,
// stride kLaStride; the lower triangle is read).  Each panel of 8 columns is
// factored by wave 0 in registers (lane = row; pivots and multipliers taken
// from their lanes with readlane, 1/sqrt by a hardware estimate and two
// Newton steps); the trailing lower tiles are then updated by all four waves on
// the FP64 matrix cores (16x16x4, K = 8).  On return the LDS matrix is L
// (zero above the diagonal) and sm[S_INVD + k] = 1 / L_kk.
__device__ inline void cholesky_lds(double *La, double *sm, int q, int lane) {
  for (int kb = 0; kb < 8; ++kb) {
    const int k0 = 8 * kb;
    if (q == 0) {
      double v[8];
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) v[jj] = lane >= k0 ? La[lane * kLaStride + k0 + jj] : 0.0;
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        const int k = k0 + jj;
        const double d = bcast_lane(v[jj], k);
        const double il = rsq_nr(d, 2);
        v[jj] = lane > k ? v[jj] * il : (lane == k ? d * il : 0.0);
        if (lane == 0) sm[S_INVD + k] = il;
#pragma unroll
        for (int j2 = jj + 1; j2 < 8; ++j2) v[j2] = fma(-v[jj], bcast_lane(v[jj], k0 + j2), v[j2]);
      }
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) La[lane * kLaStride + k0 + jj] = v[jj];
    }
    __syncthreads();
    if (kb == 7) break;
    // A[i][j] -= sum over the panel of L[i][k] L[j][k] for i, j >= s: the lower
    // 16x16 tiles that reach past s, dealt to the waves in turn
    const int s = k0 + 8, t0 = s >> 4;
    const int c16 = lane & 15, k4 = lane >> 4;
    int t = 0;
    for (int I = t0; I < 4; ++I)
      for (int J = t0; J <= I; ++J, ++t) {
        if ((t & 3) != q) continue;
        f64x4 acc;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc[r] = La[(16 * I + Mfma<double>::row(lane, r)) * kLaStride + 16 * J + c16];
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
          const int kc = k0 + 4 * kk + k4;
          acc = Mfma<double>::mac(-La[(16 * I + c16) * kLaStride + kc], La[(16 * J + c16) * kLaStride + kc],
                                  acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * I + Mfma<double>::row(lane, r), j = 16 * J + c16;
          if (i >= s && j >= s) La[i * kLaStride + j] = acc[r];
        }
      }
    __syncthreads();
  }
}

// Solve L L^T w = b with the factor in LDS (b in sm[S_VEC], w into sm[S_WV]):
// column-oriented forward and backward substitution in wave 0, lane = row.
__device__ inline void cholesky_solve_lds(const double *La, double *sm, int q, int lane) {
  if (q != 0) return;
  double z = sm[S_VEC + lane];
#pragma unroll 8
  for (int k = 0; k < 64; ++k) {
    const double zk = bcast_lane(z, k) * sm[S_INVD + k];
    const double l = La[lane * kLaStride + k];
    z = lane == k ? zk : (lane > k ? fma(-l, zk, z) : z);
  }
#pragma unroll 8
  for (int k = 63; k >= 0; --k) {
    const double wk = bcast_lane(z, k) * sm[S_INVD + k];
    const double l = La[k * kLaStride + lane];
    z = lane == k ? wk : (lane < k ? fma(-l, wk, z) : z);
  }
  sm[S_WV + lane] = z;
}

// Rotation of one pair: zero the inner product gam of columns with squared
// norms alp, bet.  t = sign(z) / (|z| + sqrt(1 + z^2)), z = (bet - alp) /
// (2 gam), from the hardware reciprocal and square root (t only steers
// convergence; a large |z| gives t -> 0, the right limit); c = (1 + t^2)^{-1/2}
// in FP64 from that t, so (c, s = c t) is orthogonal to working precision.
// Pairs with a relative inner product below 1e-30 are left alone: their
// rotation would not change a column by one FP64 unit.
__device__ inline void rotation(double alp, double bet, double gam, double &cs, double &sn,
                                double &tg, double &off) {
  off = fabs(gam) * rsq_nr(alp * bet, 0);  // a convergence measure: the estimate suffices
  const float z = (float)((bet - alp) * __builtin_amdgcn_rcp(2.0 * gam));
  const float az = fabsf(z);
  const float tf =
      copysignf(__builtin_amdgcn_rcpf(az + __builtin_amdgcn_sqrtf(fmaf(az, az, 1.0f))), z);
  const bool on = off > 1e-30;  // branch-free: the select drops the NaN of gam = 0
  const double t = on ? (double)tf : 0.0;
  const double c0 = rsq_nr(fma(t, t, 1.0), 2);
  cs = on ? c0 : 1.0;
  sn = cs * t;
  tg = t * gam;
}

// One round of 8 pairs (A[j], B[j]) of this wave; the norms of pair j's
// columns at nrm[ia], nrm[ib] of group j's lanes (LDS, this wave's slots), read
// before the inner products are summed so that their latency overlaps.
// x_p <- c x_p - s x_q, x_q <- s x_p + c x_q.
template <typename PA, typename PB>
__device__ inline void jacobi_round(PA pa, PB pb, int ia, int ib, double *nrm, double tol, int rid,
                                    int &hi, int r) {
  const double alp = nrm[ia], bet = nrm[ib];
  const double gam = group_sums8([&](int j) { return pa(j) * pb(j); }, r);
  double cs, sn, tg, off;
  rotation(alp, bet, gam, cs, sn, tg, off);
  hi = off > tol ? rid : hi;
  if ((r & 7) == 0) {
    nrm[ia] = alp - tg;
    nrm[ib] = bet + tg;
  }
  // every lane of group j holds pair j's rotation: read it from lane 8 j
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const double c_ = bcast_lane(cs, 8 * j), s_ = bcast_lane(sn, 8 * j);
    const double xp = pa(j), xq = pb(j);
    pa(j) = fma(c_, xp, -s_ * xq);
    pb(j) = fma(s_, xp, c_ * xq);
  }
  wave_sync();
}

// Move the blocks to the next block-round of the 8-block round robin (block
// slot 0 fixed, slots 1..7 rotate): X of wave q <- X of wave q-1 (wave 1:
// Y of wave 0), Y of wave q <- Y of wave q+1 (wave 3: its own X); norms
// travel with their blocks.
__device__ inline void exchange_blocks(double X[8], double Y[8], double *sm, double *xch, int q,
                                       int r) {
  double *nrm = sm + S_NRM + q * 16;
  // (the previous move ended with a barrier after its last read of the area)
  // phase 1: every X, and the norms of both blocks
#pragma unroll
  for (int j = 0; j < 8; ++j) xch[(q * 8 + j) * 64 + r] = X[j];
  if (r < 16) sm[S_XN + q * 16 + r] = nrm[r];
  __syncthreads();
  double oldX[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) oldX[j] = X[j];
  if (q >= 2) {
#pragma unroll
    for (int j = 0; j < 8; ++j) X[j] = xch[((q - 1) * 8 + j) * 64 + r];
  }
  __syncthreads();
  // phase 2: every Y
#pragma unroll
  for (int j = 0; j < 8; ++j) xch[(q * 8 + j) * 64 + r] = Y[j];
  __syncthreads();
  if (q == 1) {
#pragma unroll
    for (int j = 0; j < 8; ++j) X[j] = xch[(0 * 8 + j) * 64 + r];
  }
  if (q <= 2) {
#pragma unroll
    for (int j = 0; j < 8; ++j) Y[j] = xch[((q + 1) * 8 + j) * 64 + r];
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) Y[j] = oldX[j];
  }
  // norms: X slots 0..7, Y slots 8..15
  if (r < 8) {
    const double *xn = sm + S_XN;
    nrm[r] = q == 0 ? xn[r] : (q == 1 ? xn[0 * 16 + 8 + r] : xn[(q - 1) * 16 + r]);
  } else if (r < 16) {
    const double *xn = sm + S_XN;
    nrm[r] = q <= 2 ? xn[(q + 1) * 16 + r] : xn[q * 16 + (r - 8)];
  }
  __syncthreads();
}

// Column at slot i of round t of the round robin on 8 (slot 0 fixed, slots
// 1..7 rotate); round t pairs slots (u, 7 - u), u < 4.
__host__ __device__ constexpr int intra_slot(int t, int i) {
  return i == 0 ? 0 : ((i - 1 - t + 70) % 7) + 1;
}

__device__ inline int wave_max_int(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// One-sided Jacobi on the distributed factor: per sweep, the 7 rounds of
// pairs inside each block, then 7 block-rounds of 8 rounds pairing X[j] with
// Y[(j + t) mod 8].  The pairing repeats every 63 rounds, so any 63
// consecutive rounds meet every pair once: the rotations stop at the first
// block move after which 63 rounds have passed without a pair above tol
// (relative inner product |x_p.x_q| / (|x_p| |x_q|) measured before its
// rotation).  The blocks may then sit away from their home slots, which only
// relabels the eigenpairs; with `home` the remaining block moves of the sweep
// bring every block back (column k at slot k again).  Returns the sweeps
// begun, negative when max_sweeps sweeps did not converge.
__device__ inline int jacobi_dist(double X[8], double Y[8], double *sm, double *xch,
                                  double tol, int max_sweeps, bool home, int q, int r) {
  double *nrm = sm + S_NRM + q * 16;
  const int g = r >> 3, gu = g & 3, gy = g < 4 ? 0 : 8;
  int rounds = 0, hi = 0, ck = 0, sweep = 0, moves = 0;
  bool done = false;
  while (!done && sweep < max_sweeps) {
    ++sweep;
    // Fresh squared norms each sweep: the running update alp - t gam is exact
    // only for the exact angle, and its drift would steer the rotations of
    // nearly equal columns (a degenerate cluster) instead of their inner
    // products, stalling convergence.
    {
      const double a = group_sums8([&](int j) { return X[j] * X[j]; }, r);
      const double b = group_sums8([&](int j) { return Y[j] * Y[j]; }, r);
      if ((r & 7) == 0) {
        nrm[r >> 3] = a;
        nrm[8 + (r >> 3)] = b;
      }
      wave_sync();
    }
#pragma unroll
    for (int t = 0; t < 7; ++t) {
      // groups 0..3: pairs inside X; groups 4..7: the same pairs inside Y
      jacobi_round(
          [&](int j) -> double & { return j < 4 ? X[intra_slot(t, j)] : Y[intra_slot(t, j - 4)]; },
          [&](int j) -> double & {
            return j < 4 ? X[intra_slot(t, 7 - j)] : Y[intra_slot(t, 7 - (j - 4))];
          },
          gy + intra_slot(t, gu), gy + intra_slot(t, 7 - gu), nrm, tol, ++rounds, hi, r);
    }
    for (moves = 0; moves < 7 && !done; ++moves) {
#pragma unroll
      for (int t = 0; t < 8; ++t)
        jacobi_round([&](int j) -> double & { return X[j]; },
                     [&](int j) -> double & { return Y[(j + t) & 7]; }, g, 8 + ((g + t) & 7), nrm,
                     tol, ++rounds, hi, r);
      // post this wave's last round above tol; the block move's barriers
      // publish it (two slots by parity: a slot is rewritten only after the
      // next move, which every wave passes after reading it)
      const int w = wave_max_int(hi);
      double *slot = sm + S_MAX + (ck & 1) * 4;
      if (r == 0) slot[q] = (double)w;
      exchange_blocks(X, Y, sm, xch, q, r);
      const int last = max(max((int)slot[0], (int)slot[1]), max((int)slot[2], (int)slot[3]));
      ++ck;
      done = rounds - last >= 63;
    }
  }
  if (home)
    for (; moves < 7; ++moves) exchange_blocks(X, Y, sm, xch, q, r);
  return done ? sweep : -sweep;
}

// Load the columns this wave holds of the FP64 matrix in LDS (lane = row).
__device__ inline void load_dist(const double *M, double X[8], double Y[8], int q, int r) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    X[j] = M[r * kLaStride + pos_x(q, j)];
    Y[j] = M[r * kLaStride + pos_y(q, j)];
  }
}

// The 10 upper 16x16 tiles of a symmetric 64x64 product, dealt to the four
// waves: wave q takes tiles t = q, q + 4, q + 8.
__device__ inline void tile_of(int t, int &I, int &J) {
  int a = 0, b = 0, n = 0;
  for (int x = 0; x < 4; ++x)
    for (int y = x; y < 4; ++y) {
      if (n == t) {
        a = x;
        b = y;
      }
      ++n;
    }
  I = a;
  J = b;
}

// C = M^T M (K x 64 operand M, rows of stride ld) on the matrix cores: this
// wave's share of the upper tiles.
template <typename T>
__device__ inline void syrk_share(const T *M, int ld, int ksteps, typename Mfma<T>::V acc[3], int q,
                                  int lane) {
  const int c16 = lane & 15, k4 = lane >> 4;
  int oi[3], oj[3];
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    acc[u] = Mfma<T>::zero();
    int I, J;
    // waves 2 and 3 hold two tiles: their third repeats the first and is
    // not stored, so the loop carries no branch
    tile_of(q + 4 * u < 10 ? q + 4 * u : q, I, J);
    oi[u] = 16 * I + c16;
    oj[u] = 16 * J + c16;
  }
  const T *row0 = M + k4 * ld;
  int kk = 0;
  // four K steps a pass: every operand load issued before the products
  for (; kk + 4 <= ksteps; kk += 4) {
    T a[4][3], b[4][3];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const T *row = row0 + 4 * (kk + t) * ld;
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        a[t][u] = row[oi[u]];
        b[t][u] = row[oj[u]];
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int u = 0; u < 3; ++u) acc[u] = Mfma<T>::mac(a[t][u], b[t][u], acc[u]);
  }
  for (; kk < ksteps; ++kk) {
    const T *row = row0 + 4 * kk * ld;
#pragma unroll
    for (int u = 0; u < 3; ++u) acc[u] = Mfma<T>::mac(row[oi[u]], row[oj[u]], acc[u]);
  }
}

template <typename T>
__device__ inline void syrk_store(const typename Mfma<T>::V acc[3], T *out, int ld, T alpha, int q,
                                  int lane) {
  const int c16 = lane & 15;
  const int nt = q < 2 ? 3 : 2;
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    if (u >= nt) continue;
    int I, J;
    tile_of(q + 4 * u, I, J);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * I + Mfma<T>::row(lane, r), j = 16 * J + c16;
      const T v = alpha * acc[u][r];
      out[i * ld + j] = v;
      if (I != J) out[j * ld + i] = v;
    }
  }
}

// The same product into the FP64 LDS matrix (stride kLaStride) plus c I.
template <typename T>
__device__ inline void syrk_store_f64(const typename Mfma<T>::V acc[3], double *out, double c, int q,
                                      int lane) {
  const int c16 = lane & 15;
  const int nt = q < 2 ? 3 : 2;
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    if (u >= nt) continue;
    int I, J;
    tile_of(q + 4 * u, I, J);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * I + Mfma<T>::row(lane, r), j = 16 * J + c16;
      const double v = (double)acc[u][r] + (i == j ? c : 0.0);
      out[i * kLaStride + j] = v;
      if (I != J) out[j * kLaStride + i] = v;
    }
  }
}

// sum_j a[j] v[j] over 64 terms in FP64 (four independent chains)
template <typename TA> __device__ inline double dot64(const TA *a, const double *v) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
  for (int j = 0; j < 64; j += 4) {
    s0 = fma((double)a[j], v[j], s0);
    s1 = fma((double)a[j + 1], v[j + 1], s1);
    s2 = fma((double)a[j + 2], v[j + 2], s2);
    s3 = fma((double)a[j + 3], v[j + 3], s3);
  }
  return (s0 + s1) + (s2 + s3);
}

// ------------------------------------------- inverse square root (MFMA)
// Column block of an FP64 64 x 64 matrix held by one wave: columns
// 16 q .. 16 q + 15 as four 16x16 accumulator tiles of the FP64 16x16x4 MFMA
// (tile I, element r: row 16 I + lane / 16 + 4 r, column 16 q + lane % 16).
// The same registers are the right operand of that MFMA: at K step kk it
// reads rows 4 kk + lane / 16, which is element kk % 4 of tile kk / 4.
typedef f64x4 ColBlock[4];

// C = M B for the wave's column block: M (left operand) from LDS, row-major
// with stride kLaStride; B and C column blocks in registers.
__device__ inline void mm_colblock(const double *M, const ColBlock &B, ColBlock &C, int lane) {
  const int c16 = lane & 15, k4 = lane >> 4;
#pragma unroll
  for (int I = 0; I < 4; ++I) C[I] = Mfma<double>::zero();
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const double b = B[kk >> 2][kk & 3];
#pragma unroll
    for (int I = 0; I < 4; ++I)
      C[I] = Mfma<double>::mac(M[(16 * I + c16) * kLaStride + 4 * kk + k4], b, C[I]);
  }
}

__device__ inline void store_colblock(double *M, const ColBlock &B, int q, int lane) {
#pragma unroll
  for (int I = 0; I < 4; ++I)
#pragma unroll
    for (int r = 0; r < 4; ++r) M[(16 * I + (lane >> 4) + 4 * r) * kLaStride + 16 * q + (lane & 15)] = B[I][r];
}

__device__ inline double sum4(const double *v) { return (v[0] + v[1]) + (v[2] + v[3]); }

// Products of symmetric iterates by tiles: wave q forms the tiles (I, q) of
// its column block for I = q, q + 1 (mod 4), and, for the two waves rot and
// rot + 1, also I = q + 2, storing each with its mirror (q, I).  Any rot gives
// the ten tiles of the upper triangle once: (q, q + 1) for every q, and the
// two pairs two apart from the waves rot and rot + 1.  Those two waves form
// three tiles, the others two; rot moves that extra tile between waves (and
// so between SIMDs) without changing the count.
struct SymTiles {
  int I[3];   // tile rows
  int n;      // tiles stored
};
__device__ inline SymTiles sym_tiles(int q, int rot) {
  return SymTiles{{q, (q + 1) & 3, (q + 2) & 3}, ((q - rot) & 3) < 2 ? 3 : 2};
}

// C[t] = rows I[t] of M times the column block B (NT 16 x 16 tiles).
template <int NT>
__device__ inline void mm_tiles_n(const double *M, const ColBlock &B, const SymTiles &st, f64x4 C[3], int lane) {
  const int c16 = lane & 15, k4 = lane >> 4;
  const double *r[NT];
#pragma unroll
  for (int t = 0; t < 3; ++t) C[t] = Mfma<double>::zero();  // an unformed tile reads as zero
#pragma unroll
  for (int t = 0; t < NT; ++t) r[t] = M + (16 * st.I[t] + c16) * kLaStride + k4;
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const double b = B[kk >> 2][kk & 3];
#pragma unroll
    for (int t = 0; t < NT; ++t) C[t] = Mfma<double>::mac(r[t][4 * kk], b, C[t]);
  }
}

// This wave's tiles (three or two; one branch outside the product).
__device__ inline void mm_tiles3(const double *M, const ColBlock &B, const SymTiles &st, f64x4 C[3], int lane) {
  if (st.n == 3)
    mm_tiles_n<3>(M, B, st, C, lane);
  else
    mm_tiles_n<2>(M, B, st, C, lane);
}

// Store the stored tiles of C (scaled by sc) and their mirrors.
__device__ inline void store_tiles3(double *M, const f64x4 C[3], const SymTiles &st, double sc, int q, int lane) {
  const int c = 16 * q + (lane & 15), k4 = lane >> 4;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    if (t >= st.n) break;
    const int I = st.I[t];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * I + k4 + 4 * r;
      const double v = sc * C[t][r];
      M[row * kLaStride + c] = v;
      if (I != q) M[c * kLaStride + row] = v;
    }
  }
}

__device__ inline void load_colblock(const double *M, ColBlock &B, int q, int lane) {
#pragma unroll
  for (int I = 0; I < 4; ++I)
#pragma unroll
    for (int r = 0; r < 4; ++r) B[I][r] = M[(16 * I + (lane >> 4) + 4 * r) * kLaStride + 16 * q + (lane & 15)];
}

struct IsqrtStatus {
  int iters;       // products of the iteration taken (negative: no convergence)
  bool finite;
  double s;        // the scale: Z ~ (A / s)^{-1/2}
};

// Z = (A / s)^{-1/2} of the SPD matrix A in LDS (row-major, stride kLaStride,
// both triangles, every eigenvalue >= lmin > 0) by the scaled coupled
// Newton-Schulz iteration (Higham, Numer. Algorithms 15, 1997; Functions of
// Matrices, 2008, ch. 6):
//     T_k = (3 I - a_k Z_k Y_k) / 2,  Y_{k+1} = sqrt(a_k) Y_k T_k,
//     Z_{k+1} = sqrt(a_k) T_k Z_k,    Y_0 = A / s, Z_0 = I,
// s = ||A||_F >= lambda_max.  Every Z_k Y_k is a polynomial in A whose
// eigenvalues lie in [l_k, 1]; the step maps mu -> a mu (3 - a mu)^2 / 4,
// and a_k = 3 / (1 + sqrt(l_k) + l_k) gives the two ends of the interval the
// same image (l_{k+1}), so l_k grows by up to 27/4 a step while far from 1
// and converges quadratically near it; a_k -> 1 there.  Z and Y are carried
// as separate products (the coupled form is numerically stable; folding
// Y = A Z is not).  Z Y and the new Y and Z are symmetric polynomials in A:
// with SYM (FP32 mode) each is formed on ten of its sixteen 16 x 16 tiles and
// mirrored, three eighths less matrix-core work a step.  Z Y and Y T take the
// three-tile roles on the waves rot, rot + 1 and T Z on the other two, so the
// pair Y T, T Z (between the same two barriers) costs every wave five tiles;
// rot is chosen per work item so that two work items sharing a CU put their
// three-tile waves of Z Y on different SIMDs.  At the FP32-mode
// tolerance W then stays within 4e-9 of the eigendecomposition's on the
// steady-state 80 x 80 matrices, as with full products (the stopping rule
// sets the error); at FP64 tolerances the mirroring costs up to two digits,
// so FP64 mode forms every product in full (W within 2e-13).  Mirroring also
// lets the two iterates drift apart as A grows ill-conditioned (the rounding
// of Y and Z no longer commutes): FP32 mode forms every product in full too
// once l_0 = lmin / s is below kNsMirrorMinL.  The iteration stops once the
// predicted residual after the step, 3/4 ||a_k Z_k Y_k - I||_F^2, is <= tol.
// On return Z is in Zc (this wave's column block) and in Zb (LDS); A's area
// (Yb) has been overwritten.  Every wave takes the same decisions (the
// residual is summed over the workgroup).
//
// kNsMirrorMinL: with FP32 state the mirrored iterates track the full ones
// up to condition numbers of A~ near 2e4 (l_0 ~ 5e-5) and fall behind by
// 3.7e4 (2e-3 from the oracle against 3e-4); 1e-4 keeps a factor of two.
constexpr double kNsMirrorMinL = 1e-4;

// The iteration of ns_isqrt from its scale s and l = lmin / s, with Yc the
// column block q of A (read by the prologue).
template <bool SYM>
__device__ inline IsqrtStatus ns_iterate(double *Yb, double *Zb, double *sm, double s, double l, double tol,
                                         int max_it, ColBlock &Yc, ColBlock &Zc, int q, int lane, int rot) {
  const int col = 16 * q + (lane & 15), k4 = lane >> 4;
  ColBlock Tc;
  // k = 0 (Z_0 = I): T_0 = (3 I - a A / s) / 2, Z_1 = sqrt(a) T_0,
  // Y_1 = sqrt(a) / s A T_0 (A read from LDS)
  double al = 3.0 / (1.0 + sqrt(l) + l);
  double sa = sqrt(al);
#pragma unroll
  for (int I = 0; I < 4; ++I)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const bool dg = 16 * I + k4 + 4 * r == col;
      Tc[I][r] = 0.5 * ((dg ? 3.0 : 0.0) - (al / s) * Yc[I][r]);
      Zc[I][r] = sa * Tc[I][r];
    }
  f64x4 Yt[3], Zt[3];        // tiled form: this wave's tiles of the new Y and Z
  const SymTiles st = sym_tiles(q, rot), stz = sym_tiles(q, rot + 2);
  double ysc = sa / s, zsc = 1.0;  // their scales, applied when stored
  if constexpr (SYM) {
    mm_tiles3(Yb, Tc, st, Yt, lane);
  } else {
    mm_colblock(Yb, Tc, Yc, lane);
#pragma unroll
    for (int I = 0; I < 4; ++I) Yc[I] *= sa / s;
  }
  l = al * l * (3.0 - al * l) * (3.0 - al * l) * 0.25;
  int it = 1;
  bool conv = false, finite = true;
  for (;;) {
    __syncthreads();  // every read of Yb and Zb of the last step is done
    if constexpr (SYM) {
      if (!conv) store_tiles3(Yb, Yt, st, ysc, q, lane);
      if (it == 1)
        store_colblock(Zb, Zc, q, lane);  // Z_1 = sqrt(a) T_0, formed in full
      else
        store_tiles3(Zb, Zt, stz, zsc, q, lane);
      __syncthreads();
      if (!conv) load_colblock(Yb, Yc, q, lane);
      load_colblock(Zb, Zc, q, lane);
    } else {
      if (!conv) store_colblock(Yb, Yc, q, lane);
      store_colblock(Zb, Zc, q, lane);
      __syncthreads();
    }
    if (conv || !finite || it >= max_it) break;
    al = 3.0 / (1.0 + sqrt(l) + l);
    sa = sqrt(al);
    double e2 = 0.0;
    if constexpr (SYM) {
      // P = Z Y on this wave's tiles; T = (3 I - a P) / 2 there, mirrored
      f64x4 Pt[3];
      mm_tiles3(Zb, Yc, st, Pt, lane);
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const double wgt = t >= st.n ? 0.0 : (st.I[t] == q ? 1.0 : 2.0);  // mirrors count twice
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double d = 16 * st.I[t] + k4 + 4 * r == col ? 1.0 : 0.0;
          const double e = fma(al, Pt[t][r], -d);
          e2 = fma(wgt * e, e, e2);
          Pt[t][r] = d - 0.5 * e;
        }
      }
      e2 = wave_sum(e2);
      if (lane == 0) sm[S_RES + q] = e2;
      __syncthreads();  // every read of Zb (as Z) is done
      store_tiles3(Zb, Pt, st, 1.0, q, lane);
      __syncthreads();
      load_colblock(Zb, Tc, q, lane);
    } else {
      mm_colblock(Zb, Yc, Tc, lane);  // P = Z Y
#pragma unroll
      for (int I = 0; I < 4; ++I)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double d = 16 * I + k4 + 4 * r == col ? 1.0 : 0.0;
          const double e = fma(al, Tc[I][r], -d);  // a P - I
          e2 = fma(e, e, e2);
          Tc[I][r] = d - 0.5 * e;                  // (3 I - a P) / 2
        }
      e2 = wave_sum(e2);
      if (lane == 0) sm[S_RES + q] = e2;
      __syncthreads();  // every read of Zb (as Z) is done
      store_colblock(Zb, Tc, q, lane);
      __syncthreads();
    }
    const double d2 = sum4(sm + S_RES);
    finite = isfinite(d2);
    conv = finite && 0.75 * d2 <= tol;
    if constexpr (SYM) {
      if (!conv) mm_tiles3(Yb, Tc, st, Yt, lane);  // Y T (the last step needs only Z)
      mm_tiles3(Zb, Zc, stz, Zt, lane);            // T Z
      ysc = zsc = sa;
    } else {
      ColBlock Zn;
      if (!conv) mm_colblock(Yb, Tc, Yc, lane);
      mm_colblock(Zb, Zc, Zn, lane);
#pragma unroll
      for (int I = 0; I < 4; ++I) {
        Yc[I] *= sa;
        Zc[I] = Zn[I] * sa;
      }
    }
    l = al * l * (3.0 - al * l) * (3.0 - al * l) * 0.25;
    ++it;
  }
  return IsqrtStatus{conv ? it : -it, finite, s};
}

template <bool SYM>
__device__ inline IsqrtStatus ns_isqrt(double *Yb, double *Zb, double *sm, double lmin, double tol,
                                       int max_it, ColBlock &Zc, int q, int lane, int rot) {
  const int col = 16 * q + (lane & 15), k4 = lane >> 4;
  ColBlock Yc;
  double ss = 0.0;
#pragma unroll
  for (int I = 0; I < 4; ++I)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double v = Yb[(16 * I + k4 + 4 * r) * kLaStride + col];
      Yc[I][r] = v;
      ss = fma(v, v, ss);
    }
  ss = wave_sum(ss);
  if (lane == 0) sm[S_RES + q] = ss;
  __syncthreads();
  const double s = sqrt(sum4(sm + S_RES));
  const double l = lmin / s;
  if constexpr (SYM) {
    if (l >= kNsMirrorMinL) return ns_iterate<true>(Yb, Zb, sm, s, l, tol, max_it, Yc, Zc, q, lane, rot);
  }
  return ns_iterate<false>(Yb, Zb, sm, s, l, tol, max_it, Yc, Zc, q, lane, rot);
}

// The same iteration in FP32 on the FP32 matrix cores (twice the FP64 rate).
// Column blocks as FP32 16x16x4 accumulator tiles (tile I, element r: row
// 16 I + 4 (lane / 16) + r, column 16 q + lane % 16); FP32 matrices in LDS
// with row stride kNs32Stride (left-operand reads fall in distinct banks).
constexpr int kNs32Stride = 68;
constexpr int kNsGOff = 3 * 64 * kNs32Stride;  // G after the three FP32 iterates (floats)
typedef f32x4 ColBlock32[4];

// 4 x 4 transpose of (lane group, register): out[g][i] = in[i][g] for the
// four 16-lane groups g; v_permlane32_swap exchanges bit 1 of the two indices,
// v_permlane16_swap bit 0.  Applied to one accumulator tile (element (4 g + r,
// c) in lane (g, c), register r) it gives the right-operand form of the FP32
// MFMA, whose step kk reads element (4 kk + g, c) in lane (g, c).
__device__ inline f32x4 tile_to_rhs(f32x4 v) {
  auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[0]), __float_as_uint(v[2]), false, false);
  auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[1]), __float_as_uint(v[3]), false, false);
  auto c = __builtin_amdgcn_permlane16_swap(a[0], b[0], false, false);
  auto d = __builtin_amdgcn_permlane16_swap(a[1], b[1], false, false);
  return f32x4{__uint_as_float(c[0]), __uint_as_float(c[1]), __uint_as_float(d[0]), __uint_as_float(d[1])};
}

// C = M B for the wave's column block, with the contraction index permuted:
// step kk of lane group g takes k = 16 g + kk (the sum is over all 64 k in
// any order), so each lane's left operand of a tile is 16 consecutive floats
// of one row (four 16-byte LDS reads, all issued before the products), and
// its right operand is row 16 g + kk of the column block: element kk % 4 of
// tile g in lane group kk / 4, a (lane group, tile) transpose per register.
__device__ inline void mm_colblock32(const float *M, const ColBlock32 &B, ColBlock32 &C, int lane) {
  const int c16 = lane & 15, g = lane >> 4;
  f32x4 Av[4][4];
#pragma unroll
  for (int I = 0; I < 4; ++I)
#pragma unroll
    for (int t = 0; t < 4; ++t)
      Av[I][t] = *(const f32x4 *)(M + (16 * I + c16) * kNs32Stride + 16 * g + 4 * t);
  f32x4 Bt[4];  // Bt[a][r]: step 4 a + r
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const f32x4 v = tile_to_rhs(f32x4{B[0][r], B[1][r], B[2][r], B[3][r]});
#pragma unroll
    for (int a = 0; a < 4; ++a) Bt[a][r] = v[a];
  }
#pragma unroll
  for (int I = 0; I < 4; ++I) C[I] = Mfma<float>::zero();
#pragma unroll
  for (int kk = 0; kk < 16; ++kk)
#pragma unroll
    for (int I = 0; I < 4; ++I) C[I] = Mfma<float>::mac(Av[I][kk >> 2][kk & 3], Bt[kk >> 2][kk & 3], C[I]);
  // issue order: the 16 LDS reads, the transposes, then the 64 products
  __builtin_amdgcn_sched_group_barrier(0x100, 16, 0);
  __builtin_amdgcn_sched_group_barrier(0x002, 64, 0);
  __builtin_amdgcn_sched_group_barrier(0x008, 64, 0);
}

__device__ inline void store_colblock32(float *M, const ColBlock32 &B, int q, int lane) {
#pragma unroll
  for (int I = 0; I < 4; ++I)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      M[(16 * I + 4 * (lane >> 4) + r) * kNs32Stride + 16 * q + (lane & 15)] = B[I][r];
}

// ns_isqrt in FP32 for A = c I + G, with G (FP32, in LDS) exact: the Gram of
// the FP32 products.  Three FP32 areas hold Y, Z and T; T gets its own so that
// it is written as soon as it is formed, Z is overwritten once the products
// that read it are done, and Y (read only by the second pair of products)
// after the next barrier: two barriers a step.  The residual is summed in
// FP64.
__device__ inline IsqrtStatus ns_isqrt32(const float *G, float *Yb, float *Zb, float *Tb, double *sm,
                                         double c, double tol, int max_it, ColBlock32 &Zc, int q, int lane) {
  const int col = 16 * q + (lane & 15), g4 = 4 * (lane >> 4);
  ColBlock32 Yc, Tc;
  double ss = 0.0;
#pragma unroll
  for (int I = 0; I < 4; ++I)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float v = G[(16 * I + g4 + r) * kNs32Stride + col];
      const double a = (double)v + (16 * I + g4 + r == col ? c : 0.0);
      Yc[I][r] = v;
      ss = fma(a, a, ss);
    }
  ss = wave_sum(ss);
  if (lane == 0) sm[S_RES + q] = ss;
  __syncthreads();
  const double s = sqrt(sum4(sm + S_RES));
  double l = c / s;
  // k = 0 (Z_0 = I): T_0 = (3 I - a A / s) / 2, Z_1 = sqrt(a) T_0,
  // Y_1 = sqrt(a) / s (G T_0 + c T_0)
  double al = 3.0 / (1.0 + sqrt(l) + l);
  float sa = (float)sqrt(al);
  const float as = (float)(al / s), cf = (float)c;
#pragma unroll
  for (int I = 0; I < 4; ++I)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const bool dg = 16 * I + g4 + r == col;
      Tc[I][r] = 0.5f * ((dg ? 3.0f : 0.0f) - as * (Yc[I][r] + (dg ? cf : 0.0f)));
      Zc[I][r] = sa * Tc[I][r];
    }
  mm_colblock32(G, Tc, Yc, lane);
  const float ys = (float)(sqrt(al) / s);
#pragma unroll
  for (int I = 0; I < 4; ++I) Yc[I] = (Yc[I] + Tc[I] * cf) * ys;
  l = al * l * (3.0 - al * l) * (3.0 - al * l) * 0.25;
  store_colblock32(Yb, Yc, q, lane);
  store_colblock32(Zb, Zc, q, lane);
  __syncthreads();
  int it = 1;
  bool conv = false, finite = true;
  while (it < max_it) {
    al = 3.0 / (1.0 + sqrt(l) + l);
    sa = (float)sqrt(al);
    const float alf = (float)al;
    mm_colblock32(Zb, Yc, Tc, lane);  // P = Z Y
    double e2 = 0.0;
#pragma unroll
    for (int I = 0; I < 4; ++I)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float d = 16 * I + g4 + r == col ? 1.0f : 0.0f;
        const float e = fmaf(alf, Tc[I][r], -d);  // a P - I
        e2 = fma((double)e, (double)e, e2);
        Tc[I][r] = d - 0.5f * e;                  // (3 I - a P) / 2
      }
    e2 = wave_sum(e2);
    if (lane == 0) sm[S_RES + q] = e2;
    store_colblock32(Tb, Tc, q, lane);
    __syncthreads();  // T complete; every read of Zb is done
    const double d2 = sum4(sm + S_RES);
    finite = isfinite(d2);
    conv = finite && 0.75 * d2 <= tol;
    ColBlock32 Zn;
    if (!conv) mm_colblock32(Yb, Tc, Yc, lane);  // Y T (the last step needs only Z)
    mm_colblock32(Tb, Zc, Zn, lane);             // T Z
#pragma unroll
    for (int I = 0; I < 4; ++I) Zc[I] = Zn[I] * sa;
    store_colblock32(Zb, Zc, q, lane);
    __syncthreads();  // Z complete; every read of Yb and Tb is done
    l = al * l * (3.0 - al * l) * (3.0 - al * l) * 0.25;
    ++it;
    if (conv || !finite) break;
#pragma unroll
    for (int I = 0; I < 4; ++I) Yc[I] *= sa;
    store_colblock32(Yb, Yc, q, lane);  // read after the next barrier
  }
  return IsqrtStatus{conv ? it : -it, finite, s};
}

// Row i of M x (M: 64 x 64 FP32 in LDS, row stride kNs32Stride; x: FP64 in
// LDS) for i = 16 q + lane / 4: four lanes a row, 16 terms each, summed over
// the quad (the result is in all four lanes).
__device__ inline double matvec_quad(const float *M, const double *x, int q, int lane) {
  const int i = 16 * q + (lane >> 2), t = lane & 3;
  const float *mr = M + i * kNs32Stride + 16 * t;
  const double *xr = x + 16 * t;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
  for (int j = 0; j < 16; j += 4) {
    s0 = fma((double)mr[j], xr[j], s0);
    s1 = fma((double)mr[j + 1], xr[j + 1], s1);
    s2 = fma((double)mr[j + 2], xr[j + 2], s2);
    s3 = fma((double)mr[j + 3], xr[j + 3], s3);
  }
  double v = (s0 + s1) + (s2 + s3);
  v += dpp_f64<0xB1>(v);  // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);  // quad_perm [2,3,0,1]
  return v;
}

// ------------------------------------------- P-form inverse square root
// The scaled Newton-Schulz iteration written on P_k = Z_k Y_k alone: with
// T_k = (3 I - a_k P_k) / 2 (a polynomial in P_k, so all these matrices
// commute), Z_{k+1} = sqrt(a_k) T_k Z_k gives
//     P_{k+1} = a_k P_k T_k^2 = a_k (9/4 P_k - 3/2 a_k P_k^2 + 1/4 a_k^2 P_k^3),
// P_0 = A~ / s, and Z = prod_k sqrt(a_k) T_k -> (A~ / s)^{-1/2}.  Two products
// of one symmetric matrix with its own powers a step (P^2, then P^2 P), each
// on the ten upper 16 x 16 tiles: a rounding error of P_k is a slightly
// different symmetric P_k, which the iteration carries to I like any other,
// so no product of two separately rounded iterates is ever mirrored.  Z is
// never formed: the rows the update needs are carried instead,
//     V_{k+1} = sqrt(a_k) V_k T_k,  V_0 = X' (owned rows x members),
// so V_final = X' Z and X' W = sqrt(c / s) V, and the mean weights through
//     h_{k+1} = sqrt(a_k) T_k h_k,  h_0 = b:  X' w = X' Z^2 b / s = V h / s.
// A rounding error delta of P_k enters Z as delta / mu where mu is the
// eigenvalue it perturbs; the smallest eigenvalues are of order l_k, so the
// steps with l_k small carry the cancellation.  MIXED (FP32 handles): P is
// updated in FP64 until l_k >= kNspSwitch, then in FP32: P_{k+1} is stored
// in FP32 from l_k = 0.01 on, when its own bound l_{k+1} is 0.059 or more,
// so its rounding enters Z at 1e-6 at most.  The FP32 Gram already perturbs
// the smallest eigen-directions by about eps32 times the condition number
// kappa of A~, and l_0 = lambda_min / ||A~||_F <= 1 / kappa: the FP32 steps
// add a few percent to the Gram's error.  (The mean weights Z^2 b lean on
// the smallest eigenvalues: a switch at 1e-3 saves one more FP64 step but
// adds a quarter to the error of the analysis mean.)
//
// Storage: P and P^2 as full 64 x 64 matrices (both triangles; FP64 with row
// stride kLaStride, or FP32 with row stride kNs32Stride in the FP32 steps,
// in the same two areas), V in place of the owned patch rows ([row][member],
// row stride kXsStride, element type of the handle).  Each wave keeps the
// column block q of P in registers (the right operand of every product and
// the column block q of T).
constexpr double kNspSwitch = 0.01;

// Tile I of a column block held in registers, I a runtime value (selects,
// so that the block stays in registers).
__device__ __forceinline__ f64x4 cb_tile(const ColBlock &B, int I) {
  return I == 0 ? B[0] : I == 1 ? B[1] : I == 2 ? B[2] : B[3];
}
__device__ __forceinline__ f32x4 cb_tile32(const ColBlock32 &B, int I) {
  return I == 0 ? B[0] : I == 1 ? B[1] : I == 2 ? B[2] : B[3];
}

// FP32 matrices (row stride kNs32Stride): the FP32 accumulator layout is
// tile J, element r: row 16 J + 4 (lane / 16) + r; as the right operand with
// the contraction order k = 16 J + 4 (lane / 16) + r at step 4 J + r, the
// left operand of a lane is four consecutive floats of one row per J.
__device__ __forceinline__ void f32_load_colblock(const float *M, ColBlock32 &B, int q, int lane) {
  const int c16 = lane & 15, g4 = 4 * (lane >> 4);
#pragma unroll
  for (int J = 0; J < 4; ++J)
#pragma unroll
    for (int r = 0; r < 4; ++r) B[J][r] = M[(16 * J + g4 + r) * kNs32Stride + 16 * q + c16];
}

// Store tile (I, q) (FP32 accumulator layout) and its mirror.
__device__ __forceinline__ void f32_store_tile(float *M, int I, int q, const f32x4 &v, int lane) {
  const int c16 = lane & 15, g4 = 4 * (lane >> 4);
#pragma unroll
  for (int r = 0; r < 4; ++r) M[(16 * I + g4 + r) * kNs32Stride + 16 * q + c16] = v[r];
  if (I != q) *(f32x4 *)(M + (16 * q + c16) * kNs32Stride + 16 * I + g4) = v;
}

// Store tile (I, q) (FP64 accumulator layout) into an FP64 matrix (row stride
// kLaStride) or, with F32, an FP32 one, with its mirror.
template <bool F32>
__device__ __forceinline__ void store_tile64(void *Mv, int I, int q, const f64x4 &v, int lane) {
  const int c16 = lane & 15, g = lane >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 16 * I + g + 4 * r;
    if constexpr (F32) {
      float *M = (float *)Mv;
      M[row * kNs32Stride + 16 * q + c16] = (float)v[r];
      if (I != q) M[(16 * q + c16) * kNs32Stride + row] = (float)v[r];
    } else {
      double *M = (double *)Mv;
      M[row * kLaStride + 16 * q + c16] = v[r];
      if (I != q) M[(16 * q + c16) * kLaStride + row] = v[r];
    }
  }
}

struct NspStatus {
  int iters;   // steps taken (negative: no convergence)
  bool finite;
  double s;    // the scale: Z ~ (A~ / s)^{-1/2}
};

struct NspState {
  double l, sc;   // lower bound of the spectrum of P_k; P_k = sc x (stored matrix)
  int it;         // steps taken
  bool conv, finite;
};

// NT tiles (rows (q + t) & 3) of M B: M an FP64 matrix in LDS (stride
// kLaStride) as the left operand, B a column block in registers, the FP64
// order (step kk takes k = 4 kk + lane / 16); all tiles in one pass over K
// so that the matrix cores always have an independent product to issue.
template <int NT>
__device__ __forceinline__ void mm_rows64(const double *M, const ColBlock &B, f64x4 C[3], int q, int lane) {
  const int c16 = lane & 15, g = lane >> 4;
  const double *r[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) r[t] = M + (16 * ((q + t) & 3) + c16) * kLaStride + g;
#pragma unroll
  for (int t = 0; t < 3; ++t) C[t] = Mfma<double>::zero();
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const double b = B[kk >> 2][kk & 3];
#pragma unroll
    for (int t = 0; t < NT; ++t) C[t] = Mfma<double>::mac(r[t][4 * kk], b, C[t]);
  }
}

// The same with FP32 matrices on the FP32 matrix cores (FP32 order).
template <int NT>
__device__ __forceinline__ void mm_rows32(const float *M, const ColBlock32 &B, f32x4 C[3], int q, int lane) {
  const int c16 = lane & 15, g4 = 4 * (lane >> 4);
  const float *r[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) r[t] = M + (16 * ((q + t) & 3) + c16) * kNs32Stride + g4;
#pragma unroll
  for (int t = 0; t < 3; ++t) C[t] = Mfma<float>::zero();
#pragma unroll
  for (int J = 0; J < 4; ++J) {
    f32x4 a[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) a[t] = *(const f32x4 *)(r[t] + 16 * J);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr)
#pragma unroll
      for (int t = 0; t < NT; ++t) C[t] = Mfma<float>::mac(a[t][rr], B[J][rr], C[t]);
  }
}

// V T for the member block q: ncb row tiles of V (rows 16 cb + .., element
// type TV, row stride kXsStride) times T's column block q, T = 3/2 I - ta Pc
// formed from the registers.  FP64 order with an FP64 column block (F32
// false), FP32 order on the FP32 matrix cores otherwise.
template <typename TV, bool F32, typename CB>
__device__ __forceinline__ void v_times_t(const TV *V, const CB &Pc, double ta, int ncb, f64x4 Vo[4], int q,
                                          int lane) {
  const int c16 = lane & 15, g = lane >> 4;
  if constexpr (F32) {
    ColBlock32 Tc;
#pragma unroll
    for (int J = 0; J < 4; ++J)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        Tc[J][r] = ((16 * J + 4 * g + r) == (16 * q + c16) ? 1.5f : 0.0f) - (float)ta * Pc[J][r];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      if (cb < ncb) {
        const TV *vr = V + (16 * cb + c16) * kXsStride + 4 * g;
        f32x4 acc = Mfma<float>::zero();
#pragma unroll
        for (int J = 0; J < 4; ++J)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc = Mfma<float>::mac((float)vr[16 * J + r], Tc[J][r], acc);
        Vo[cb] = f64x4{acc[0], acc[1], acc[2], acc[3]};
      }
    }
  } else {
    ColBlock Tc;
#pragma unroll
    for (int J = 0; J < 4; ++J)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        Tc[J][r] = ((16 * J + g + 4 * r) == (16 * q + c16) ? 1.5 : 0.0) - ta * (double)Pc[J][r];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      if (cb < ncb) {
        const TV *vr = V + (16 * cb + c16) * kXsStride + g;
        f64x4 acc = Mfma<double>::zero();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) acc = Mfma<double>::mac((double)vr[4 * kk], Tc[kk >> 2][kk & 3], acc);
        Vo[cb] = acc;
      }
    }
  }
}

// (M h)_i for row i = 16 q + c16 of a symmetric matrix M in LDS (FP64, row
// stride kLaStride, or with F32 FP32, stride kNs32Stride): lane group g sums
// the columns 16 g .. 16 g + 15, rows_sum adds the four groups.
template <bool F32>
__device__ __forceinline__ double row_dot(const void *Mv, const double *hb, int i, int g) {
  double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
  if constexpr (F32) {
    const float *pr = (const float *)Mv + i * kNs32Stride + 16 * g;
#pragma unroll
    for (int j = 0; j < 16; j += 4) {
      const f32x4 v = *(const f32x4 *)(pr + j);
      p0 = fma((double)v[0], hb[16 * g + j], p0);
      p1 = fma((double)v[1], hb[16 * g + j + 1], p1);
      p2 = fma((double)v[2], hb[16 * g + j + 2], p2);
      p3 = fma((double)v[3], hb[16 * g + j + 3], p3);
    }
  } else {
    const double *pr = (const double *)Mv + i * kLaStride + 16 * g;
#pragma unroll
    for (int j = 0; j < 16; j += 4) {
      p0 = fma(pr[j], hb[16 * g + j], p0);
      p1 = fma(pr[j + 1], hb[16 * g + j + 1], p1);
      p2 = fma(pr[j + 2], hb[16 * g + j + 2], p2);
      p3 = fma(pr[j + 3], hb[16 * g + j + 3], p3);
    }
  }
  return rows_sum((p0 + p1) + (p2 + p3));
}

// V M for the member block q: ncb row tiles of V times the column block q of
// the symmetric matrix M in LDS (FP64 order, or FP32 order and storage with
// F32), as v_times_t forms V T.
template <typename TV, bool F32>
__device__ __forceinline__ void v_times_m(const TV *V, const void *Mv, int ncb, f64x4 Wo[4], int q, int lane) {
  const int c16 = lane & 15, g = lane >> 4;
  if constexpr (F32) {
    ColBlock32 B;
    f32_load_colblock((const float *)Mv, B, q, lane);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      if (cb < ncb) {
        const TV *vr = V + (16 * cb + c16) * kXsStride + 4 * g;
        f32x4 acc = Mfma<float>::zero();
#pragma unroll
        for (int J = 0; J < 4; ++J)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc = Mfma<float>::mac((float)vr[16 * J + r], B[J][r], acc);
        Wo[cb] = f64x4{acc[0], acc[1], acc[2], acc[3]};
      }
    }
  } else {
    ColBlock B;
    load_colblock((const double *)Mv, B, q, lane);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      if (cb < ncb) {
        const TV *vr = V + (16 * cb + c16) * kXsStride + g;
        f64x4 acc = Mfma<double>::zero();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) acc = Mfma<double>::mac((double)vr[4 * kk], B[kk >> 2][kk & 3], acc);
        Wo[cb] = acc;
      }
    }
  }
}

// One step of the P-form iteration with P held in FP64 (Pd; P^2 in Qd) or,
// with F32, in FP32 (the same areas as float).  Forms T_k applied to V and h
// and P^2 before the first barrier, stores V and h after it (every read of
// them came before) with P_{k+1} (to FP32 storage when TO32).  Returns
// whether P_{k+1} went to FP32.
template <typename TV, bool F32>
__device__ __forceinline__ bool nsp_step(double *Pd, double *Qd, TV *V, int ncb, double *hb, double *sm,
                                         double tol, double tol2, int max_it, bool may32, NspState &S, int q,
                                         int lane, int rot) {
  // (the lane index made opaque a step: the lane-dependent diagonal selects
  // and addresses are formed where used rather than hoisted out of the step
  // loops, where the two loops of the mixed form would hold both sets)
  asm volatile("" : "+v"(lane));
  const int c16 = lane & 15, g = lane >> 4;
  const int n1 = ((q - rot) & 3) < 2 ? 3 : 2, n2 = ((q - rot - 2) & 3) < 2 ? 3 : 2;  // tiles of P^2, of P^3
  const double al = 3.0 / (1.0 + sqrt(S.l) + S.l), sa = sqrt(al);
  const double ta = 0.5 * al;   // T = 3/2 I - ta P (P true, scale applied)
  float *P32 = (float *)Pd, *Q32 = (float *)Qd;
  using CB = typename std::conditional<F32, ColBlock32, ColBlock>::type;
  using QV = typename std::conditional<F32, f32x4, f64x4>::type;
  CB Pc;
  double e2 = 0.0;
  if constexpr (F32) {
    f32_load_colblock(P32, Pc, q, lane);
#pragma unroll
    for (int J = 0; J < 4; ++J)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double d = fma(al, (double)Pc[J][r], (16 * J + 4 * g + r) == (16 * q + c16) ? -1.0 : 0.0);
        e2 = fma(d, d, e2);
      }
  } else {
    load_colblock(Pd, Pc, q, lane);
#pragma unroll
    for (int J = 0; J < 4; ++J) {
      Pc[J] *= S.sc;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double d = fma(al, Pc[J][r], (16 * J + g + 4 * r) == (16 * q + c16) ? -1.0 : 0.0);
        e2 = fma(d, d, e2);
      }
    }
  }
  e2 = wave_sum_dpp(e2);
  if (lane == 0) sm[S_RES + q] = e2;
  // V T_k (member block q of every row block)
  f64x4 Vo[4];
  v_times_t<TV, F32, CB>(V, Pc, ta, ncb, Vo, q, lane);
  // h: sqrt(a) (3/2 h - ta P h) for row 16 q + c16 (segment g, summed over lanes)
  const int hi = 16 * q + c16;
  const double th = fma(-ta, row_dot<F32>(F32 ? (const void *)P32 : (const void *)Pd, hb, hi, g) * S.sc, 1.5 * hb[hi]);
  // P^2 on this wave's tiles (q + t, q), t < n1 (not needed after the last step)
  const bool more = S.it + 1 < max_it;
  if (more) {
    QV Qo[3];
    if constexpr (F32) {
      if (n1 == 3) mm_rows32<3>(P32, Pc, Qo, q, lane); else mm_rows32<2>(P32, Pc, Qo, q, lane);
#pragma unroll
      for (int t = 0; t < 3; ++t)
        if (t < n1) f32_store_tile(Q32, (q + t) & 3, q, Qo[t], lane);
    } else {
      if (n1 == 3) mm_rows64<3>(Pd, Pc, Qo, q, lane); else mm_rows64<2>(Pd, Pc, Qo, q, lane);
#pragma unroll
      for (int t = 0; t < 3; ++t)
        if (t < n1) store_tile64<false>(Qd, (q + t) & 3, q, Qo[t] * S.sc, lane);
    }
  }
  __syncthreads();  // #1: P^2 and the residual complete; every read of P, V and h done
  const double d2 = sum4(sm + S_RES);
  S.finite = isfinite(d2);
  S.conv = S.finite && 0.75 * d2 <= tol;
  // second-order finish when the residual is below tol2 (P^2 is at hand):
  // sqrt(a) (I - E/2 + 3/8 E^2), E = a P - I, in place of sqrt(a) T = sqrt(a)
  // (I - E/2); with V T and T h known it is sqrt(a) (5/2 X T - 15/8 X + 3/8
  // a^2 X P^2) for X = V, h.  Its truncation, about 5/16 |E|^3, stays under
  // the rounding the handle's precision leaves
  const bool fin2 = S.finite && !S.conv && more && 0.75 * d2 <= tol2;
  ++S.it;
  bool went32 = false;
  if (fin2) {
    f64x4 W2[4];
    v_times_m<TV, F32>(V, F32 ? (const void *)Q32 : (const void *)Qd, ncb, W2, q, lane);
    const double q2 = row_dot<F32>(F32 ? (const void *)Q32 : (const void *)Qd, hb, hi, g);
    const double hold = hb[hi];
    f64x4 Vold[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      if (cb < ncb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * cb + (F32 ? 4 * g + r : g + 4 * r);
          Vold[cb][r] = (double)V[row * kXsStride + 16 * q + c16];
        }
      }
    }
    __syncthreads();  // every read of V, h and P^2 done
    const double c2 = 0.375 * al * al;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      if (cb < ncb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * cb + (F32 ? 4 * g + r : g + 4 * r);
          V[row * kXsStride + 16 * q + c16] = (TV)(sa * fma(c2, W2[cb][r], fma(2.5, Vo[cb][r], -1.875 * Vold[cb][r])));
        }
      }
    }
    if (g == 0) hb[hi] = sa * fma(c2, q2, fma(2.5, th, -1.875 * hold));
    S.conv = true;
  } else {
    // V <- sqrt(a) V T_k (this wave's members), h <- its update
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      if (cb < ncb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * cb + (F32 ? 4 * g + r : g + 4 * r);
          V[row * kXsStride + 16 * q + c16] = (TV)(sa * Vo[cb][r]);
        }
      }
    }
    if (g == 0) hb[hi] = sa * th;
  }
  if (!S.conv && S.finite && more) {
    // P_{k+1} = a (9/4 P - 3/2 a P^2 + 1/4 a^2 P^3) on the tiles (q + t, q),
    // t < n2 (the other role assignment), P^3 = P^2 P, P^2 read back;
    // written over P (no wave reads P after the first barrier)
    QV Ro[3];
    if constexpr (F32) {
      if (n2 == 3) mm_rows32<3>(Q32, Pc, Ro, q, lane); else mm_rows32<2>(Q32, Pc, Ro, q, lane);
      const float alf = (float)al;
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        if (t < n2) {
          const int I = (q + t) & 3;
          const f32x4 pv = cb_tile32(Pc, I);
          f32x4 Pn;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float qv = Q32[(16 * I + 4 * g + r) * kNs32Stride + 16 * q + c16];
            Pn[r] = alf * (2.25f * pv[r] - 1.5f * alf * qv + 0.25f * alf * alf * Ro[t][r]);
          }
          f32_store_tile(P32, I, q, Pn, lane);
        }
      }
    } else {
      if (n2 == 3) mm_rows64<3>(Qd, Pc, Ro, q, lane); else mm_rows64<2>(Qd, Pc, Ro, q, lane);
      went32 = may32 && S.l >= kNspSwitch;
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        if (t < n2) {
          const int I = (q + t) & 3;
          const f64x4 pv = cb_tile(Pc, I);
          f64x4 Pn;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const double qv = Qd[(16 * I + g + 4 * r) * kLaStride + 16 * q + c16];
            Pn[r] = al * (2.25 * pv[r] - 1.5 * al * qv + 0.25 * al * al * Ro[t][r]);
          }
          if (went32)
            store_tile64<true>(Pd, I, q, Pn, lane);
          else
            store_tile64<false>(Pd, I, q, Pn, lane);
        }
      }
    }
  }
  __syncthreads();  // #2: P_{k+1}, V and h complete
  S.sc = 1.0;
  S.l = al * S.l * (3.0 - al * S.l) * (3.0 - al * S.l) * 0.25;
  return went32;
}

// The P-form iteration on A~ (FP64, full, in area0; area1 the second
// area) with V_0 = X' in V (owned rows x members, row stride kXsStride, ncb
// row blocks) and h_0 = b in hb[0..63].  On return V holds V_final = X' Z
// and hb h_final = Z b.  Every wave takes the same decisions (the residual
// is summed over the workgroup).
template <typename TV, bool MIXED>
__device__ __forceinline__ NspStatus nsp_isqrt(double *area0, double *area1, TV *V, int ncb, double *hb,
                                               double *sm, double c, double tol, int max_it, int q, int lane,
                                               int rot) {
  // s = ||A~||_F
  {
    double ss = 0.0;
    const int col = 16 * q + (lane & 15), g = lane >> 4;
#pragma unroll
    for (int I = 0; I < 4; ++I)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double v = area0[(16 * I + g + 4 * r) * kLaStride + col];
        ss = fma(v, v, ss);
      }
    ss = wave_sum(ss);
    if (lane == 0) sm[S_RES + q] = ss;
  }
  __syncthreads();
  const double s = sqrt(sum4(sm + S_RES));
  NspState S{c / s, 1.0 / s, 0, false, true};
  // threshold of the second-order finish: with FP32 state the rounding keeps
  // the result near 1e-6 whatever the truncation below it, so sqrt(tol) (the
  // residual at 1e-3: a step earlier on the 80x80 domains, no loss); in FP64
  // tol^(2/3) keeps its truncation, about 5/16 |E|^3, where the first-order
  // finish at tol leaves its own, 3/8 |E|^2
  const double tol2 = sizeof(TV) == 4 ? sqrt(tol) : cbrt(tol * tol);
  bool to32 = false;
  for (;;) {
    to32 = nsp_step<TV, false>(area0, area1, V, ncb, hb, sm, tol, tol2, max_it, MIXED, S, q, lane, rot);
    if (S.conv || !S.finite || S.it >= max_it || to32) break;
  }
  if constexpr (MIXED) {
    if (to32 && !S.conv && S.finite && S.it < max_it) {
      for (;;) {
        nsp_step<TV, true>(area0, area1, V, ncb, hb, sm, tol, tol2, max_it, false, S, q, lane, rot);
        if (S.conv || !S.finite || S.it >= max_it) break;
      }
    }
  }
  return NspStatus{S.conv ? S.it : -S.it, S.finite, s};
}


// Stages 1-6 of one work item, shared by the analysis and its adjoint.  On
// return: the forecast patch in xs (rows = patch nodes, lane = member) with its
// member means in xm, the scaled innovation in dd, the slope means in yb, the
// weights sqrt(g) in sg, w in sm[S_WV], lambda in sm[S_LAMV], the factor
// U = L J of the Jacobi (lane = row) in X / Y, and W (row-major, stride
// kYsStride) at the start of the U area.
struct CoreStatus {
  bool bad, conv, lam_ok;
  int sweeps;  // Jacobi sweeps begun
};

// The bank noise of stage 1, member by member (lane = patch row): wave q
// loads V[r][k] for its members k = q, q + 4, ... (bank_load, issued with the
// rows' loads) and adds vs V to xs[r][k] once the rows are in LDS (bank_add).
// One member's values lie in a small window of one screen, a few cache lines
// per load, where a row of all members touches a line per member.  Member
// k's draw is read from lane k.
template <typename T>
__device__ __forceinline__ void bank_load(const AnaArgs<T> &A, const InstDesc &in, const int *pn,
                                          const BankDraw &bd, T val[16], int np, int q, int lane) {
  const int m = in.m, rc = lane < np ? lane : 0;
  const int ij = pn[64 + rc], ri = ij & 0xFFFF, rj = ij >> 16;
  const int side = in.bank_side, mask = side - 1;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int k = q + 4 * t, kc = k < m ? k : 0;
    const int64_t base = ((int64_t)__builtin_amdgcn_readlane((int)(bd.base >> 32), kc) << 32) |
                         (uint32_t)__builtin_amdgcn_readlane((int)bd.base, kc);
    const int oy = __builtin_amdgcn_readlane(bd.oy, kc), ox = __builtin_amdgcn_readlane(bd.ox, kc);
    const int orient = __builtin_amdgcn_readlane(bd.orient, kc);
    int u = (orient & 1) ? rj : ri;
    int v = (orient & 1) ? ri : rj;
    if (orient & 2) u = -u;
    if (orient & 4) v = -v;
    val[t] = (T)A.bank[base + (int64_t)((oy + u) & mask) * side + ((ox + v) & mask)];
  }
}

template <typename T>
__device__ __forceinline__ void bank_add(const InstDesc &in, const T val[16], T vs, T *xs, int np, int q,
                                         int lane, int r_lo) {
  const int m = in.m;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int k = q + 4 * t;
    if (k < m && lane >= r_lo && lane < np) xs[lane * kXsStride + k] = fma_t(vs, val[t], xs[lane * kXsStride + k]);
  }
}

// Stage 1's patch rows of X_b = a X_a + V (+ a2 X_a(k-1)): xs[r][member] for
// this wave's rows r = q, q + 4, ... (up to 16).  Rows and members are
// clamped to valid ones so that every load is issued unconditionally, back
// to back; the values of clamped rows are not stored, those of members past
// m are stored as zero.  With BANK the noise is loaded by bank_load along
// with the rows and added by bank_add once the rows are in LDS.
template <typename T, bool FUSED, bool BANK, bool PREV>
__device__ __forceinline__ void stage_rows(const AnaArgs<T> &A, const InstDesc &in, const int *pn,
                                           const BankDraw &bd, T a, T a2, T vs, T *xs, int np, int q,
                                           int lane, int r_lo) {
  const int m = in.m, ln = lane < m ? lane : 0;
  T bv[16];
  if constexpr (BANK) bank_load<T>(A, in, pn, bd, bv, np, q, lane);  // in flight with the rows
  for (int r0 = r_lo + q; r0 < np; r0 += 16 * kWaves) {
    T xv[16], pv[16], nv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int r = r0 + u * kWaves, rc = r < np ? r : 0;
      const int64_t e = in.x_off + (int64_t)pn[rc] * m + ln;
      xv[u] = A.x_in[e];
      if constexpr (PREV) pv[u] = A.x_prev[e];
      if constexpr (FUSED && !BANK) nv[u] = A.v_in[e];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int r = r0 + u * kWaves;
      if (r >= np) continue;
      T v = xv[u];
      if constexpr (FUSED) {
        T noise = BANK ? (T)0 : vs * nv[u];
        if constexpr (PREV) noise = fma_t(a2, pv[u], noise);  // the AR(2) term joins the noise
        v = fma_t(a, xv[u], noise);
      }
      xs[r * kXsStride + lane] = lane < m ? v : (T)0;
    }
  }
  if constexpr (BANK) {
    __syncthreads();
    bank_add<T>(in, bv, vs, xs, np, q, lane, r_lo);
  }
}

// Stage 1's patch rows r_lo .. n_patch - 1 of X_b (every choice of noise
// source and history); the caller brackets it with barriers.
template <typename T, bool FUSED>
__device__ __forceinline__ void stage_patch_rows(const AnaArgs<T> &A, const InstDesc &in, const int *pn,
                                                 const BankDraw &bd, T *xs, int np, int q, int lane, int r_lo) {
  const bool use_bank = FUSED && A.noise_bank;
  const bool use_prev = FUSED && A.x_prev && in.a2 != 0.0;
  const T a = (T)in.a, a2 = (T)in.a2, vs = (T)in.vscale;
  if (!FUSED)
    stage_rows<T, false, false, false>(A, in, pn, bd, a, a2, vs, xs, np, q, lane, r_lo);
  else if (use_bank)
    use_prev ? stage_rows<T, true, true, true>(A, in, pn, bd, a, a2, vs, xs, np, q, lane, r_lo)
             : stage_rows<T, true, true, false>(A, in, pn, bd, a, a2, vs, xs, np, q, lane, r_lo);
  else
    use_prev ? stage_rows<T, true, false, true>(A, in, pn, bd, a, a2, vs, xs, np, q, lane, r_lo)
             : stage_rows<T, true, false, false>(A, in, pn, bd, a, a2, vs, xs, np, q, lane, r_lo);
}

// Stages 1-3: on return A~ = c I + Yt^T Yt (FP64, both triangles) at the start
// of the U area, b = Yt^T sqrt(g) d in sm[S_VEC]; returns whether an
// observation was not finite.  CL (covariance localisation): stages 1-2 only,
// without the taper on the observation weights and without the slope operand.
template <typename T, bool FUSED, bool G32 = false, bool CL = false>
__device__ __forceinline__ bool stage_gram(const AnaArgs<T> &A, const DomItem &it, const InstDesc &in,
                                           uint32_t frame, unsigned char *smem) {
  const int tid = threadIdx.x;
  const int q = tid >> 6, lane = tid & 63;
  const int m = in.m;
  const int np = it.n_patch, nobs = it.n_obs;
  const int p = 2 * nobs, p4 = (p + 3) & ~3;

  T *xs = (T *)(smem + A.off_xs);
  T *xm = (T *)(smem + A.off_xm);
  double *sg = (double *)(smem + A.off_sg);
  double *dd = (double *)(smem + A.off_dd);
  T *yb = (T *)(smem + A.off_yb);
  int *pn = (int *)(smem + A.off_pn);
  double *sm = (double *)(smem + A.off_s);
  unsigned char *U = smem + A.off_u;

  // ---- 1. node patch of X_b (rows dealt to the four waves) ----
  // patch node of row `lane` and its grid coordinates (pn[64 + r]: i | j << 16)
  const bool use_bank = FUSED && A.noise_bank;
  // closed loop: the command u_{k-2} at the patch nodes (uc, after pn)
  T *uc = (T *)(pn + kPnU);
  const bool use_u = in.model == 1 && A.u_prev2;
  if (q == 0) {
    const int g = lane < np ? A.patch_node[it.patch_off + lane] : 0;
    pn[lane] = g;
    if (use_bank) pn[64 + lane] = A.node_ij[2 * (in.node_off + g)] | (A.node_ij[2 * (in.node_off + g) + 1] << 16);
    uc[lane] = use_u && lane < np ? A.u_prev2[in.node_off + g] : (T)0;
  }
  BankDraw bd{};
  if (use_bank) bd = bank_draw(in, frame, lane < m ? lane : 0);  // lanes past m: member 0's (not stored)
  __syncthreads();
  // every row of the wave in one pass (up to 16), its loads issued back to
  // back (the choices of noise source and history are made outside the loop:
  // a load behind a branch is waited for before the next is issued)
  stage_patch_rows<T, FUSED>(A, in, pn, bd, xs, np, q, lane, 0);
  __syncthreads();
  if (tid < np) {
    T s = (T)0;
    for (int j = 0; j < m; ++j) s += xs[tid * kXsStride + j];
    xm[tid] = s / (T)m;
  }
  __syncthreads();

  // ---- 2. local slopes, weights and innovation ----
  int bad = 0;
  if (tid < nobs) {
    const uint32_t cw = A.obs_corner[it.obs_off + tid];
    ((uint32_t *)pn)[kPnCw + tid] = cw;  // kept for the slope operand below
    const int k = A.obs_sub[it.obs_off + tid];
    const int ca = cw & 255, cb = (cw >> 8) & 255, cc = (cw >> 16) & 255, cd = cw >> 24;
    const T ybx = (T)0.5 * ((xm[cb] - xm[ca]) + (xm[cd] - xm[cc]));
    const T yby = (T)0.5 * ((xm[cc] - xm[ca]) + (xm[cd] - xm[cb]));
    const double f = (!CL && in.taper_c > 0.0) ? gaspari_cohn(A.obs_dist[it.obs_off + tid] / in.taper_c) : 1.0;
    const double rx = A.r_diag[in.y_off + k], ry = A.r_diag[in.y_off + in.n_subaps + k];
    const double sgx = f / sqrt(in.r_scale * rx), sgy = f / sqrt(in.r_scale * ry);
    const double yx = (double)A.y[in.y_off + k], yy = (double)A.y[in.y_off + in.n_subaps + k];
    bad = !(isfinite(yx) && isfinite(yy));
    // predicted slopes D x_b, less D N u_{k-2} in the closed loop (N = I)
    double ypx = (double)ybx, ypy = (double)yby;
    if (use_u) {
      ypx -= 0.5 * (((double)uc[cb] - (double)uc[ca]) + ((double)uc[cd] - (double)uc[cc]));
      ypy -= 0.5 * (((double)uc[cc] - (double)uc[ca]) + ((double)uc[cd] - (double)uc[cb]));
    }
    sg[tid] = sgx;
    sg[nobs + tid] = sgy;
    dd[tid] = sgx * (yx - ypx);
    dd[nobs + tid] = sgy * (yy - ypy);
    yb[tid] = ybx;
    yb[nobs + tid] = yby;
  }
  bad = __syncthreads_or(bad);
  if constexpr (CL) return bad != 0;
  T *ys = (T *)(smem + A.off_ys);  // [p4][kYsStride], K-major MFMA operand
#pragma unroll 3
  for (int o = q; o < nobs; o += kWaves) {
    const uint32_t cw = ((const uint32_t *)pn)[kPnCw + o];
    const int ca = cw & 255, cb = (cw >> 8) & 255, cc = (cw >> 16) & 255, cd = cw >> 24;
    const T pa = xs[ca * kXsStride + lane], pb = xs[cb * kXsStride + lane];
    const T pc = xs[cc * kXsStride + lane], pd = xs[cd * kXsStride + lane];
    const T sx = (T)0.5 * ((pb - pa) + (pd - pc)) - yb[o];
    const T sy = (T)0.5 * ((pc - pa) + (pd - pb)) - yb[nobs + o];
    ys[o * kYsStride + lane] = lane < m ? (T)sg[o] * sx : (T)0;
    ys[(nobs + o) * kYsStride + lane] = lane < m ? (T)sg[nobs + o] * sy : (T)0;
  }
  for (int o = p + q; o < p4; o += kWaves) ys[o * kYsStride + lane] = (T)0;
  __syncthreads();
  {  // b = Y^T sqrt(g) d, member = lane (p4 - p rows of ys are zero): wave q
     // sums the row quads 4 q, 4 q + 16, ... into sm[S_VEC + 64 q] (free
     // until the transform), wave 0 adds the four after the Gram's barrier
    double b0 = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0;
    for (int s = 4 * q; s < p4; s += 16) {
      b0 = fma((double)ys[s * kYsStride + lane], s < p ? dd[s] : 0.0, b0);
      b1 = fma((double)ys[(s + 1) * kYsStride + lane], s + 1 < p ? dd[s + 1] : 0.0, b1);
      b2 = fma((double)ys[(s + 2) * kYsStride + lane], s + 2 < p ? dd[s + 2] : 0.0, b2);
      b3 = fma((double)ys[(s + 3) * kYsStride + lane], s + 3 < p ? dd[s + 3] : 0.0, b3);
    }
    sm[S_VEC + 64 * q + lane] = (b0 + b1) + (b2 + b3);
  }

  // ---- 3. Gram on the matrix cores ----
  typename Mfma<T>::V acc[3];
  syrk_share<T>(ys, kYsStride, p4 / 4, acc, q, lane);
  __syncthreads();
  if constexpr (G32) {
    // G = Yt^T Yt as the FP32 products left it (exact), row stride kNs32Stride
    syrk_store<T>(acc, (T *)U + kNsGOff, kNs32Stride, (T)1, q, lane);
  } else {
    const double c = (double)(m - 1) / in.rho;
    double *La = (double *)U;  // A~ = c I + Y^T Y in FP64, then its Cholesky factor
    syrk_store_f64<T>(acc, La, c, q, lane);
  }
  __syncthreads();
  // b's quarters summed (read first after the transform's next barrier)
  if (q == 0) sm[S_VEC + lane] = (sm[S_VEC + lane] + sm[S_VEC + 64 + lane]) +
                                 (sm[S_VEC + 128 + lane] + sm[S_VEC + 192 + lane]);
  return bad != 0;
}

template <typename T, bool FUSED>
__device__ __forceinline__ CoreStatus analysis_core(const AnaArgs<T> &A, const DomItem &it,
                                                     const InstDesc &in, uint32_t frame,
                                                     unsigned char *smem, double X[8], double Y[8]) {
  const int tid = threadIdx.x;
  const int q = tid >> 6, lane = tid & 63;
  const int m = in.m;
  double *sm = (double *)(smem + A.off_s);
  unsigned char *U = smem + A.off_u;
  double *La = (double *)U;
  const double c = (double)(m - 1) / in.rho;
  const bool bad = stage_gram<T, FUSED>(A, it, in, frame, smem);

  // ---- 4./5. FP64 Cholesky, w, one-sided Jacobi ----
  cholesky_lds(La, sm, q, lane);
  cholesky_solve_lds(La, sm, q, lane);
  load_dist(La, X, Y, q, lane);
  __syncthreads();
  // (W and the adjoint sum over all 64 eigenpairs: their order is free)
  const int sweeps = jacobi_dist(X, Y, sm, (double *)U, A.jtol, A.max_sweeps, false, q, lane);
  const bool conv = sweeps > 0;

  // ---- 6. lambda and W = sqrt(c) (U Lambda^{-3/4}) (U Lambda^{-3/4})^T ----
  column_sums(X, Y, [](double v) { return v * v; }, sm + S_LAM, q, lane);
  __syncthreads();
  const double lam_l = sm[S_LAM + lane];
  const bool lam_ok = __syncthreads_and(isfinite(lam_l) && lam_l > 0.0);
  if (q == 0) {
    sm[S_LAM + lane] = 1.0 / sqrt(lam_l * sqrt(lam_l));
    sm[S_LAMV + lane] = lam_l;
  }
  __syncthreads();
  T *ut = (T *)U;  // [64][kYsStride]: (U Lambda^{-3/4})^T, K-major
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int px = pos_x(q, j), py = pos_y(q, j);
    ut[px * kYsStride + lane] = (T)(X[j] * sm[S_LAM + px]);
    ut[py * kYsStride + lane] = (T)(Y[j] * sm[S_LAM + py]);
  }
  __syncthreads();
  typename Mfma<T>::V acc[3];
  syrk_share<T>(ut, kYsStride, 16, acc, q, lane);
  __syncthreads();
  T *wmat = ut;  // W row-major [64][kYsStride]
  syrk_store<T>(acc, wmat, kYsStride, (T)sqrt(c), q, lane);
  __syncthreads();
  return CoreStatus{bad, conv, lam_ok, sweeps > 0 ? sweeps : -sweeps};
}

// Transform of the analysis (stages 4-6): the inverse square root by the
// Newton-Schulz iteration in FP64 (default) or with FP32 iterates, or the
// symmetric eigendecomposition by the one-sided Jacobi.
constexpr int kEigNs64 = 0, kEigNs32 = 1, kEigJacobi = 2, kEigNsp = 3, kEigNspMix = 4;

template <typename T, bool FUSED, int EIG>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_analysis(const AnaArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int q = tid >> 6, lane = tid & 63;
  int item = A.order ? A.order[blockIdx.x]
                     : (A.xcd_order ? xcd_item((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x);
  item += A.item_base;
  if (item < 0 || item >= A.n_items) return;
  const DomItem it = A.items[item];
  const InstDesc in = A.inst[it.inst];
  const int m = in.m;
  const int nown = it.n_own, np = it.n_patch;
  T *xs = (T *)(smem + A.off_xs);
  T *xm = (T *)(smem + A.off_xm);
  int *pn = (int *)(smem + A.off_pn);
  double *sm = (double *)(smem + A.off_s);
  const uint32_t frame = (FUSED && A.noise_bank) ? *A.frame : 0u;
  const double c = (double)(m - 1) / in.rho;
  bool bad, conv;
  int flag;
  T wf[16];  // this wave's column block of W, right-operand layout of the update

  if constexpr (EIG == kEigNsp || EIG == kEigNspMix) {
    // ---- 1.-3. staging and the Gram; 4.-6. the P-form iteration carrying
    // V = X' Z of the owned rows (in their place) and h = Z b ----
    constexpr bool MIXED = EIG == kEigNspMix && sizeof(T) == 4;
    const bool gbad = stage_gram<T, FUSED>(A, it, in, frame, smem);
    double *area0 = (double *)(smem + A.off_u), *area1 = area0 + 64 * kLaStride;
    const int ncb = (nown + 15) >> 4;
    // V_0 = X' of the owned rows, in place (rows past n_own and members past m zero)
    for (int e = tid; e < 16 * ncb * 64; e += kThreads) {
      const int i = e >> 6, kk = e & 63;
      xs[i * kXsStride + kk] = (i < nown && kk < m) ? xs[i * kXsStride + kk] - xm[i] : (T)0;
    }
    // the three-tile roles as in ns_isqrt: a function of the item alone
    const int per = (A.n_items + 7) >> 3;
    const int rot = ((item % per) / A.round_items) & 1;
    double *hb = sm + S_VEC;  // h_0 = b
    const NspStatus st = nsp_isqrt<T, MIXED>(area0, area1, xs, ncb, hb, sm, c, A.jtol * 0.01, A.max_sweeps, q,
                                             lane, rot);
    const int nit = st.iters > 0 ? st.iters : -st.iters;
    const bool nconv = st.iters > 0;
    const int nflag = (gbad || !st.finite ? 1 : 0) | (nconv || !st.finite ? 0 : 2) | (min(nit, 255) << 8);
    const bool keep = gbad || !st.finite || !nconv;
    if (tid == 0) A.flags[item] = nflag;
    if (keep) {
      // the forecast is the result: the owned rows of X_b again (V took their place)
      __syncthreads();
      BankDraw bd{};
      if (FUSED && A.noise_bank) bd = bank_draw(in, frame, lane < m ? lane : 0);
      stage_patch_rows<T, FUSED>(A, in, pn, bd, xs, nown, q, lane, 0);
      __syncthreads();
      for (int i = q; i < nown; i += kWaves)
        if (lane < m) A.x_out[in.x_off + (int64_t)pn[i] * m + lane] = xs[i * kXsStride + lane];
      if (tid < nown && A.x_mean) {
        const T uo = (in.model == 1 && A.u_prev2) ? ((const T *)(pn + kPnU))[tid] : (T)0;
        A.x_mean[in.node_off + pn[tid]] = xm[tid] - uo;
      }
      return;
    }
    // ---- 7. x_a = x_b + X' w = x_b + V h / s, X_a = x_a 1^T + sqrt(rho c / s) V ----
    for (int i = q; i < nown; i += kWaves) {
      double v = lane < m ? (double)xs[i * kXsStride + lane] * hb[lane] : 0.0;
      v = wave_sum(v);
      if (lane == 0) sm[S_XAM + i] = (double)xm[i] + v / st.s;
    }
    __syncthreads();
    const double wsc = sqrt(in.rho * c / st.s);
    for (int i = q; i < nown; i += kWaves)
      if (lane < m)
        A.x_out[in.x_off + (int64_t)pn[i] * m + lane] = (T)(sm[S_XAM + i] + wsc * (double)xs[i * kXsStride + lane]);
    if (tid < nown && A.x_mean) {
      // the piston fit reads this mean (in the closed loop: x_a - N u_{k-2})
      const T uo = (in.model == 1 && A.u_prev2) ? ((const T *)(pn + kPnU))[tid] : (T)0;
      A.x_mean[in.node_off + pn[tid]] = (T)sm[S_XAM + tid] - uo;
    }
    return;
  } else if constexpr (EIG == kEigJacobi) {
    // ---- 1.-6. staging, Gram, Cholesky and w, Jacobi, W in LDS ----
    double X[8], Y[8];
    const CoreStatus cs = analysis_core<T, FUSED>(A, it, in, frame, smem, X, Y);
    bad = cs.bad || !cs.lam_ok;
    conv = cs.conv;
    flag = (bad ? 1 : 0) | (conv ? 0 : 2) | (min(cs.sweeps, 255) << 8);
    const T *wmat = (const T *)(smem + A.off_u);
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) wf[kk] = wmat[(4 * kk + (lane >> 4)) * kYsStride + 16 * q + (lane & 15)];
  } else {
    bad = stage_gram<T, FUSED, EIG == kEigNs32>(A, it, in, frame, smem);
    // ---- 4. Z = (A~ / s)^{-1/2} on the matrix cores (eigenvalues >= c) ----
    // ---- 5. w = A~^{-1} b = Z (Z b) / s ----
    IsqrtStatus st;
    if constexpr (EIG == kEigNs32) {
      // FP32 iterates; the exact FP32 Gram G gives A~ = c I + G for one FP64
      // refinement of w, which carries the mean: w = w0 + Z (Z (b - A~ w0)) / s
      float *Y32 = (float *)(smem + A.off_u);
      float *Z32 = Y32 + 64 * kNs32Stride, *T32 = Z32 + 64 * kNs32Stride;
      const float *G32 = Y32 + kNsGOff;
      ColBlock32 Zc;
      st = ns_isqrt32(G32, Y32, Z32, T32, sm, c, A.jtol * 0.01, A.max_sweeps, Zc, q, lane);
      const int i = 16 * q + (lane >> 2);
      const bool lead = (lane & 3) == 0;
      const double u = matvec_quad(Z32, sm + S_VEC, q, lane);
      if (lead) sm[S_COL + i] = u;
      __syncthreads();
      const double w0 = matvec_quad(Z32, sm + S_COL, q, lane) / st.s;
      if (lead) sm[S_WV + i] = w0;
      __syncthreads();
      const double r = sm[S_VEC + i] - c * w0 - matvec_quad(G32, sm + S_WV, q, lane);
      if (lead) sm[S_COL + 64 + i] = r;
      __syncthreads();
      const double u2 = matvec_quad(Z32, sm + S_COL + 64, q, lane);
      if (lead) sm[S_COL + i] = u2;
      __syncthreads();
      const double dw = matvec_quad(Z32, sm + S_COL, q, lane) / st.s;
      if (lead) sm[S_WV + i] = w0 + dw;
      const float wsc = (float)sqrt(c / st.s);
#pragma unroll
      for (int I = 0; I < 4; ++I) {
        const f32x4 bt = tile_to_rhs(Zc[I]);
#pragma unroll
        for (int r2 = 0; r2 < 4; ++r2) wf[4 * I + r2] = (T)(wsc * bt[r2]);
      }
    } else {
      double *Yb = (double *)(smem + A.off_u);  // A~, then the iteration's two matrices
      double *Zb = Yb + 64 * kLaStride;
      ColBlock Zc;
      // Work items are dealt to the XCDs in contiguous runs (xcd_item); the
      // items past the first round_items of a run start in the second
      // dispatch round and share a CU with one of the first, whose waves
      // occupy the SIMDs one place further on: rot = 1 there keeps the
      // two items' three-tile waves apart.  A function of the item alone, so
      // every launch form takes the same roundings.
      const int per = (A.n_items + 7) >> 3;
      const int rot = ((item % per) / A.round_items) & 1;
      st = ns_isqrt<sizeof(T) == 4>(Yb, Zb, sm, c, A.jtol * 0.01, A.max_sweeps, Zc, q, lane, rot);
      if (q == 0) {
        sm[S_COL + lane] = dot64(Zb + lane * kLaStride, sm + S_VEC);
        wave_sync();
        sm[S_WV + lane] = dot64(Zb + lane * kLaStride, sm + S_COL) / st.s;
      }
      // W = sqrt(c) A~^{-1/2} = sqrt(c / s) Z: this wave's members are Z's
      // column block, already in the right-operand layout of the update
      const double wsc = sqrt(c / st.s);
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) wf[kk] = (T)(wsc * Zc[kk >> 2][kk & 3]);
    }
    conv = st.iters > 0;
    flag = (bad || !st.finite ? 1 : 0) | (conv || !st.finite ? 0 : 2) |
           (min(st.iters > 0 ? st.iters : -st.iters, 255) << 8);
    bad = bad || !st.finite;
    __syncthreads();
  }

  // ---- 7. owned rows (blend: every patch row): X_a = (x_b + X' w) 1^T + sqrt(rho) X' W ----
  const bool keep_forecast = bad || !conv;
  const bool blend = in.blend != 0 && A.stage;
  const int nupd = blend ? np : nown;
  if (blend && np > nown) {
    // the rows past the owned ones shared LDS with the transform: stage them
    // again (the same arithmetic on the same inputs, so the same values)
    __syncthreads();
    BankDraw bd{};
    if (FUSED && A.noise_bank) bd = bank_draw(in, frame, lane < m ? lane : 0);
    stage_patch_rows<T, FUSED>(A, in, pn, bd, xs, np, q, lane, nown);
    __syncthreads();
  }
  if (tid == 0) A.flags[item] = flag;
  if (tid < nupd) {
    const double mu = (double)xm[tid];
    double s = mu;
    for (int k = 0; k < m; ++k) s = fma((double)xs[tid * kXsStride + k] - mu, sm[S_WV + k], s);
    sm[S_XAM + tid] = s;
    if (blend) {
      A.stage_mean[it.patch_off + tid] = keep_forecast ? mu : s;
    } else {
      // the piston fit reads this mean; in the closed loop it is the residual
      // x_a - N u_{k-2} that the slopes y_k see
      const T uo = (in.model == 1 && A.u_prev2) ? ((const T *)(pn + kPnU))[tid] : (T)0;
      if (A.x_mean) A.x_mean[in.node_off + pn[tid]] = (keep_forecast ? xm[tid] : (T)s) - uo;
    }
  }
  __syncthreads();
  const T srho = (T)sqrt(in.rho);
  const int c16 = lane & 15, k4 = lane >> 4;
  const int J = q;  // this wave's 16 members
  for (int I = 0; I * 16 < nupd; ++I) {
    typename Mfma<T>::V o = Mfma<T>::zero();
    const int ia = 16 * I + c16;
    const bool rowok = ia < nupd;
    const int iac = rowok ? ia : 0;  // loads from a valid row, the value dropped after
    const T mu = xm[iac];
    T av[16];
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {  // every load before the products
      const int k = 4 * kk + k4;
      const T v = xs[iac * kXsStride + k];
      av[kk] = (rowok && k < m) ? v - mu : (T)0;
    }
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) o = Mfma<T>::mac(av[kk], wf[kk], o);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * I + Mfma<T>::row(lane, r);
      const int j = 16 * J + c16;
      if (i < nupd && j < m) {
        const T v = keep_forecast ? xs[i * kXsStride + j] : (T)sm[S_XAM + i] + srho * o[r];
        if (blend)
          A.stage[(int64_t)(it.patch_off + i) * 64 + j] = v;
        else
          A.x_out[in.x_off + (int64_t)pn[i] * m + j] = v;
      }
    }
  }
}

// ------------------------------------------------- covariance localisation
// The localisation Sec. 4 names beside the local analysis: the prior
// covariance tapered by a Schur product.  Per domain, over its node patch,
//   P_loc = rho_xx o (kappa X'_P X'_P^T),  kappa = rho / (m - 1),
// rho_xx the Gaspari-Cohn function of the node distance over c = taper_c
// (c = 0: no taper); with the whitened local slope operator Dt (rows scaled
// by 1 / sqrt(s r)) and the whitened innovation dd,
//   B = P_loc Dt^T (patch x p),  S = Dt B + I (p x p, FP64 Cholesky),
//   K^T = S^{-1} B_own^T,
//   x_a = x_b + K dd,  X'_a = sqrt(rho) (X'_own - K Dt X'_P / 2)
// (the deterministic EnKF update of the anomalies), written to the owned
// rows.  LDS: the patch rows, then one area for X'_P^T, P_loc and S in turn
// (FP64; S as a packed lower triangle), and B, whose owned rows become the
// solve's columns (offsets from the host).
constexpr int kEigCl = kAnalysisCl;

// index of (i, j), j <= i, in a packed lower triangle
__device__ inline int tri(int i, int j) { return ((i * (i + 1)) >> 1) + j; }

constexpr int kClPanel = 8;  // columns of a Cholesky panel (covariance localisation)

// S^{-1} (S = L L^T, L packed lower with 1 / L_ii in dg) applied in place to
// the columns cb, cb + 4, ..., cb + 4 (NU - 1) of Bm (row stride ldp; those
// past nc are neither read nor written), each in one wave's registers (rows
// lane and 64 + lane): per row i, x_i = v_i / L_ii goes to every lane by
// readlane, and the column (forward) or row (backward) of L is read once for
// all the columns.  In two halves, rows below 64 in v0 and the rest in v1:
// where x_i comes from and which half changes are then fixed in each.
template <int NU>
__device__ inline void cl_solve_columns(double *Bm, const double *S, const double *dg, int cb, int nc,
                                        int ldp, int p, int lane) {
  double v0[NU], v1[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int c = cb + 4 * u;
    const double *col = Bm + (c < nc ? c : 0) * ldp;
    v0[u] = c < nc && lane < p ? col[lane] : 0.0;
    v1[u] = c < nc && lane + 64 < p ? col[lane + 64] : 0.0;
  }
  // Row i keeps its value at step i (no later step of the sweep changes it),
  // so each sweep leaves v_i and one product v_i / L_ii per row afterwards
  // gives x_i, the same product step i broadcast.
  const int ph = min(p, 64);
  const double d0 = lane < p ? dg[lane] : 0.0, d1 = lane + 64 < p ? dg[lane + 64] : 0.0;
  for (int i = 0; i < ph; ++i) {  // L y = b, rows < 64: column i of L below the diagonal
    const double inv = dg[i];
    const double l0 = lane > i && lane < p ? S[tri(lane, i)] : 0.0;
    const double l1 = lane + 64 < p ? S[tri(lane + 64, i)] : 0.0;
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const double x = bcast_lane(v0[u], i) * inv;
      v0[u] = fma(-l0, x, v0[u]);
      v1[u] = fma(-l1, x, v1[u]);
    }
  }
  for (int i = 64; i < p; ++i) {  // rows >= 64: only v1 changes
    const double inv = dg[i];
    const double l1 = lane + 64 > i && lane + 64 < p ? S[tri(lane + 64, i)] : 0.0;
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const double x = bcast_lane(v1[u], i - 64) * inv;
      v1[u] = fma(-l1, x, v1[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    v0[u] *= d0;
    v1[u] *= d1;
  }
  for (int i = p - 1; i >= 64; --i) {  // L^T x = y, rows >= 64: row i of L left of the diagonal
    const double inv = dg[i];
    const double l0 = S[tri(i, lane)];
    const double l1 = lane + 64 < i ? S[tri(i, lane + 64)] : 0.0;
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const double x = bcast_lane(v1[u], i - 64) * inv;
      v1[u] = fma(-l1, x, v1[u]);
      v0[u] = fma(-l0, x, v0[u]);
    }
  }
  for (int i = ph - 1; i >= 0; --i) {  // rows < 64: only v0 changes
    const double inv = dg[i];
    const double l0 = lane < i ? S[tri(i, lane)] : 0.0;
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const double x = bcast_lane(v0[u], i) * inv;
      v0[u] = fma(-l0, x, v0[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    v0[u] *= d0;
    v1[u] *= d1;
  }
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int c = cb + 4 * u;
    if (c < nc) {
      double *col = Bm + c * ldp;
      if (lane < p) col[lane] = v0[u];
      if (lane + 64 < p) col[lane + 64] = v1[u];
    }
  }
}

template <typename T, bool FUSED>
__global__ __launch_bounds__(kThreads) void k_analysis_cl(const AnaArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int q = tid >> 6, lane = tid & 63;
  int item = A.order ? A.order[blockIdx.x]
                     : (A.xcd_order ? xcd_item((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x);
  item += A.item_base;
  if (item < 0 || item >= A.n_items) return;
  const DomItem it = A.items[item];
  const InstDesc in = A.inst[it.inst];
  const int m = in.m, np = it.n_patch, nown = it.n_own, nobs = it.n_obs, p = 2 * nobs, ldp = p + 1;
  T *xs = (T *)(smem + A.off_xs);
  T *xm = (T *)(smem + A.off_xm);
  const double *sg = (const double *)(smem + A.off_sg);
  const double *dd = (const double *)(smem + A.off_dd);
  // corner words of the region's subapertures, as stage 2 left them
  const uint32_t *cw = (const uint32_t *)(smem + A.off_pn) + kPnCw;
  int *pn = (int *)(smem + A.off_pn);
  double *dg = (double *)(smem + A.off_s);       // pivots sqrt(S_kk) of the Cholesky
  double *xt = (double *)(smem + A.off_u);       // X'_P^T in FP64, [member][kClXtStride]
  double *Pm = (double *)(smem + A.off_u);       // P_loc [64][kLaStride], then S (packed lower)
  double *Bm = (double *)(smem + A.off_clb);     // [patch row][ldp]; rows 0..n_own the solve's columns
  const uint32_t frame = (FUSED && A.noise_bank) ? *A.frame : 0u;
  bool bad = stage_gram<T, FUSED, false, true>(A, it, in, frame, smem);

  // ---- 3. P_loc ----
  // the patch nodes' grid coordinates (stage 1 leaves them when the noise
  // comes from the bank)
  if (!(FUSED && A.noise_bank) && tid < np) {
    const int64_t g = in.node_off + pn[tid];
    pn[64 + tid] = A.node_ij[2 * g] | (A.node_ij[2 * g + 1] << 16);
  }
  for (int e = tid; e < 64 * 64; e += kThreads) {
    const int k = e >> 6, r = e & 63;
    xt[k * kClXtStride + r] = (r < np && k < m) ? (double)xs[r * kXsStride + k] - (double)xm[r] : 0.0;
  }
  __syncthreads();
  {
    // in FP64 in both precisions: the slope stencil applied to P_loc below
    // cancels most of its size (the phase is smooth), so an FP32 product's
    // rounding would come out amplified
    typename Mfma<double>::V acc[3];
    syrk_share<double>(xt, kClXtStride, 16, acc, q, lane);
    __syncthreads();
    syrk_store_f64<double>(acc, Pm, 0.0, q, lane);
  }
  __syncthreads();
  const double kap = in.rho / (double)(m - 1), cw_taper = in.taper_c;
  // one weight per pair (i >= j, the packed lower triangle's entries in
  // order), applied to both entries: P_loc and the taper are symmetric
  for (int e = tid; e < tri(np, 0); e += kThreads) {
    int i = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    i += tri(i + 1, 0) <= e ? 1 : 0;
    i -= tri(i, 0) > e ? 1 : 0;
    const int j = e - tri(i, 0);
    double t = kap;
    if (cw_taper > 0.0) {
      const int a = pn[64 + i], b = pn[64 + j];
      const double di = (double)((a & 0xFFFF) - (b & 0xFFFF)), dj = (double)((a >> 16) - (b >> 16));
      t *= gaspari_cohn(sqrt(di * di + dj * dj) / cw_taper);
    }
    Pm[i * kLaStride + j] *= t;
    if (i != j) Pm[j * kLaStride + i] *= t;
  }
  __syncthreads();

  // ---- 4. B = P_loc Dt^T ----
  for (int e = tid; e < np * p; e += kThreads) {
    const int i = e / p, s = e - i * p;
    const uint32_t w = cw[s < nobs ? s : s - nobs];
    const int ca = w & 255, cb = (w >> 8) & 255, cc = (w >> 16) & 255, cd = w >> 24;
    const double *Pi = Pm + i * kLaStride;
    const double v = s < nobs ? (Pi[cb] - Pi[ca]) + (Pi[cd] - Pi[cc]) : (Pi[cc] - Pi[ca]) + (Pi[cd] - Pi[cb]);
    Bm[i * ldp + s] = 0.5 * sg[s] * v;
  }
  __syncthreads();

  // ---- 5. S = Dt B + I, lower triangle packed, over P_loc ----
  double *S = Pm;
  for (int e = tid; e < tri(p, 0); e += kThreads) {  // the packed entries in order
    // row s of entry e: the largest s with tri(s, 0) <= e (the float root is
    // exact to one, corrected by the two comparisons)
    int s = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    s += tri(s + 1, 0) <= e ? 1 : 0;
    s -= tri(s, 0) > e ? 1 : 0;
    const int t = e - tri(s, 0);
    const uint32_t w = cw[s < nobs ? s : s - nobs];
    const int ca = w & 255, cb = (w >> 8) & 255, cc = (w >> 16) & 255, cd = w >> 24;
    const double ba = Bm[ca * ldp + t], bb = Bm[cb * ldp + t], bc = Bm[cc * ldp + t], bd = Bm[cd * ldp + t];
    const double v = s < nobs ? (bb - ba) + (bd - bc) : (bc - ba) + (bd - bb);
    S[e] = 0.5 * sg[s] * v + (s == t ? 1.0 : 0.0);
  }
  __syncthreads();
  // the solve's columns: B's owned rows (patch rows 0..n_own - 1) as they
  // stand

  // ---- 6. Cholesky S = L L^T in place (packed lower triangle), by panels
  // of kClPanel columns: wave 0 factors a panel in registers (rows k0 + lane
  // and k0 + 64 + lane; the entries of column c2 of the panel at row k0 + c2
  // come from lane c2 by readlane), then every wave subtracts the panel's
  // product from the trailing triangle: two barriers a panel (eight columns:
  // the panel's serial work, which grows with its width, against the barriers).
  // dg[k] = 1 / L_kk ----
  int fail = 0;
  for (int k0 = 0; k0 < p; k0 += kClPanel) {
    const int kb = min(kClPanel, p - k0), k1 = k0 + kb;
    if (q == 0) {
      const int r0 = k0 + lane, r1 = r0 + 64;
      double L0[kClPanel], L1[kClPanel];
#pragma unroll
      for (int c = 0; c < kClPanel; ++c) {
        L0[c] = (c < kb && r0 < p && k0 + c <= r0) ? S[tri(r0, k0 + c)] : 0.0;
        L1[c] = (c < kb && r1 < p) ? S[tri(r1, k0 + c)] : 0.0;
      }
#pragma unroll
      for (int c = 0; c < kClPanel; ++c) {
        if (c < kb) {
          const double d = bcast_lane(L0[c], c);  // the pivot (row k0 + c)
          fail |= !(d > 0.0);
          const double inv = rsq_nr(d, 2), ljj = d * inv;  // 1 / sqrt(d) refined twice
          L0[c] = lane == c ? ljj : (lane > c ? L0[c] * inv : L0[c]);
          L1[c] *= inv;
          if (lane == c) dg[k0 + c] = inv;
          // (lanes above column c2's diagonal take garbage here: never read
          // by the steps, which read a column at its diagonal and below, and
          // never stored)
#pragma unroll
          for (int c2 = c + 1; c2 < kClPanel; ++c2) {
            const double lc = bcast_lane(L0[c], c2);  // L[k0 + c2][k0 + c]
            L0[c2] = fma(-L0[c], lc, L0[c2]);
            L1[c2] = fma(-L1[c], lc, L1[c2]);
          }
        }
      }
#pragma unroll
      for (int c = 0; c < kClPanel; ++c) {
        if (c < kb && r0 < p && k0 + c <= r0) S[tri(r0, k0 + c)] = L0[c];
        if (c < kb && r1 < p) S[tri(r1, k0 + c)] = L1[c];
      }
    }
    __syncthreads();
    // trailing triangle (rows and columns from k1) on a 16 x 16 grid: the
    // panel is full (kb = kClPanel) wherever a trailing triangle is left
    for (int a = tid >> 4; a < p - k1; a += 16) {
      const int i = k1 + a;
      const double *Li = S + tri(i, k0);
      double li[kClPanel];
#pragma unroll
      for (int j = 0; j < kClPanel; ++j) li[j] = Li[j];
      for (int b = tid & 15; b <= a; b += 16) {
        const double *Lc = S + tri(k1 + b, k0);
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int j = 0; j < kClPanel; j += 2) {
          s0 = fma(li[j], Lc[j], s0);
          s1 = fma(li[j + 1], Lc[j + 1], s1);
        }
        S[tri(i, k1 + b)] -= s0 + s1;
      }
    }
    __syncthreads();
  }
  bad = bad || __syncthreads_or(fail);

  // ---- 7. K^T = S^{-1} B_own^T in place: wave q takes the columns q,
  // q + 4, ..., up to eight at a time (cl_solve_columns) ----
  const int nc = nown;
  if (!bad)
    for (int cb = q; cb < nc; cb += 4 * 8) {
      const int nu = min(8, (nc - cb + 3) >> 2);  // this wave's columns in the chunk
      if (nu <= 2)
        cl_solve_columns<2>(Bm, S, dg, cb, nc, ldp, p, lane);
      else if (nu <= 4)
        cl_solve_columns<4>(Bm, S, dg, cb, nc, ldp, p, lane);
      else if (nu <= 6)
        cl_solve_columns<6>(Bm, S, dg, cb, nc, ldp, p, lane);
      else
        cl_solve_columns<8>(Bm, S, dg, cb, nc, ldp, p, lane);
    }
  __syncthreads();
  const double *R = Bm;

  // ---- 8. M = K Dt (owned rows x patch), from each patch node's corner
  // roles: on the grid a node is corner a, b, c or d of at most one
  // subaperture each, so every observation writes its four corners' entries
  // at once (no two write the same) ----
  int *adj = (int *)dg;  // [64][4]: the subaperture where node n is corner a, b, c, d (-1: none)
  for (int e = tid; e < 64 * 4; e += kThreads) adj[e] = -1;
  __syncthreads();
  if (tid < nobs) {
    const uint32_t w = cw[tid];
#pragma unroll
    for (int t = 0; t < 4; ++t) adj[(int)((w >> (8 * t)) & 255) * 4 + t] = tid;
  }
  __syncthreads();
  double *Mk = S;  // [own row][64]
  if (!bad)
    for (int e = tid; e < nown * 64; e += kThreads) {
      const int i = e >> 6, n = e & 63;
      double v = 0.0;
      if (n < np) {
        const double *Ki = R + i * ldp;
#pragma unroll
        for (int u = 0; u < 4; ++u) {  // roles a, b, c, d
          const int o = adj[n * 4 + u];
          if (o < 0) continue;
          const double cx = (u & 1) ? 0.5 : -0.5, cy = (u & 2) ? 0.5 : -0.5;
          v = fma(Ki[o] * sg[o], cx, v);
          v = fma(Ki[nobs + o] * sg[nobs + o], cy, v);
        }
      }
      Mk[i * 64 + n] = v;
    }
  __syncthreads();

  // ---- 9. owned rows: x_a = x_b + K dd, X'_a = sqrt(rho) (X' - M X'_P / 2) ----
  if (tid == 0) A.flags[item] = bad ? 1 : 0;
  const double srho = sqrt(in.rho);
  for (int i = q; i < nown; i += kWaves) {
    const double *Ki = R + i * ldp;
    double xa = (double)xm[i];
    if (!bad) {  // K_i dd: the slopes dealt to the lanes, summed over the wave
      double part = 0.0;
      for (int s = lane; s < p; s += 64) part = fma(Ki[s], dd[s], part);
      xa += wave_sum(part);
    }
    if (lane < m) {
      double v;
      if (bad) {
        v = (double)xs[i * kXsStride + lane];
      } else {
        // M_i X'_P for this member, four partial sums
        const double *Mi = Mk + i * 64;
        double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0;
        int n = 0;
        for (; n + 3 < np; n += 4) {
          c0 = fma(Mi[n], (double)xs[n * kXsStride + lane] - (double)xm[n], c0);
          c1 = fma(Mi[n + 1], (double)xs[(n + 1) * kXsStride + lane] - (double)xm[n + 1], c1);
          c2 = fma(Mi[n + 2], (double)xs[(n + 2) * kXsStride + lane] - (double)xm[n + 2], c2);
          c3 = fma(Mi[n + 3], (double)xs[(n + 3) * kXsStride + lane] - (double)xm[n + 3], c3);
        }
        for (; n < np; ++n) c0 = fma(Mi[n], (double)xs[n * kXsStride + lane] - (double)xm[n], c0);
        const double corr = (c0 + c1) + (c2 + c3);
        v = xa + srho * (((double)xs[i * kXsStride + lane] - (double)xm[i]) - 0.5 * corr);
      }
      A.x_out[in.x_off + (int64_t)pn[i] * m + lane] = (T)v;
    }
    if (lane == 0 && A.x_mean) {
      // the piston fit reads this mean (in the closed loop: x_a - N u_{k-2})
      const T uo = (in.model == 1 && A.u_prev2) ? ((const T *)(pn + kPnU))[i] : (T)0;
      A.x_mean[in.node_off + pn[i]] = (T)xa - uo;
    }
  }
}

// ------------------------------------------------------------------ adjoint
// Reverse of one frame for the gradient of a loss of the analysis ensembles
// with respect to (rho, s, c): inflation, noise scale and taper width (Sec.
// 3.1.1 transform, Sec. 4.1 localisation, Sec. 4.2 local analyses).  Per work
// item the forward stages are recomputed by the same code, then
//   owned rows:  xa_bar = Xa_bar 1,  X'_bar = sqrt(rho) Xa_bar W + xa_bar w^T,
//                W_bar = sqrt(rho) X'^T Xa_bar,  w_bar = X'^T xa_bar;
//   w = A~^{-1} b:  b_bar = Q Lambda^{-1} Q^T w_bar,  A_bar = -b_bar w^T;
//   W = sqrt(k) A~^{-1/2}:  A_bar += sqrt(k) Q (F o (Q^T sym(W_bar) Q)) Q^T with
//                F_ij = -1 / (s_i s_j (s_i + s_j)), s = sqrt(lambda), the
//                divided differences of l^{-1/2} (its derivative on the
//                diagonal and inside degenerate clusters);
//   A~ = k I + Yt^T Yt, b = Yt^T dt:  S = sym(A_bar),
//                Yt_bar = 2 Yt S + dt b_bar^T,  dt_bar = Yt b_bar;
// and the slope-space adjoints sqrt(g) Yt_bar, sqrt(g) dt_bar go to one slot
// per (item, local slope), summed per slope by the node pass that follows.

constexpr int kQStride = 65;   // FP64 64 x 64 matrices in LDS (row stride)
// adjoint scratch (doubles)
constexpr int A_XAB = 0;       // 64: xa_bar of the owned rows
constexpr int A_WBB = 64;      // 64: w_bar
constexpr int A_TV = 128;      // 64: Lambda^{-1} Q^T w_bar
constexpr int A_BB = 192;      // 64: b_bar
constexpr int A_KAP = 256;     // 128: (df/dc) / sqrt(s r) per local slope
constexpr int A_DIN = 384;     // 128: unscaled innovation per local slope
constexpr int A_RED = 512;     // 4 waves x 8 partial sums
constexpr int A_TOTAL = 544;

// d GC / d z of the Gaspari-Cohn function above (its piecewise derivative).
__device__ inline double gaspari_cohn_dz(double z) {
  z = fabs(z);
  if (z >= 2.0) return 0.0;
  if (z <= 1.0) return (((-1.25 * z + 2.0) * z + 1.875) * z - 10.0 / 3.0) * z;
  return (((5.0 / 12.0 * z - 2.0) * z + 1.875) * z + 10.0 / 3.0) * z - 5.0 + 2.0 / (3.0 * z * z);
}

// One 16 x 16 output tile (I, J) of a 64 x 64 x 64 FP64 product on the matrix
// cores; a(i, k), b(k, j) load the operands.
template <typename FA, typename FB>
__device__ inline f64x4 mm64_tile(FA a, FB b, int I, int J, int lane) {
  const int c16 = lane & 15, k4 = lane >> 4;
  f64x4 acc = Mfma<double>::zero();
#pragma unroll 4
  for (int kk = 0; kk < 16; ++kk) {
    const int k = 4 * kk + k4;
    acc = Mfma<double>::mac(a(16 * I + c16, k), b(k, 16 * J + c16), acc);
  }
  return acc;
}

template <typename T> struct AdjArgs {
  AnaArgs<T> F;
  const T *xbar;     // adjoint of this frame's analysis ensemble [node][m]
  T *xpbar;          // out: adjoint of X' on the owned rows [node][m]
  double *xbbar;     // out: adjoint of x_b on the owned nodes [node]
  T *ybar;           // out: adjoint of Y' per (item, local slope) slot, [slot][64]
  double *dbar;      // out: adjoint of d per slot
  double *theta;     // out: (rho, s, c) adjoint per item, [item][4]
  uint32_t frame;    // frame number of the bank draws
  int32_t off_q, off_sa;
};

__device__ inline double block_sum4(double v, double *red, int slot, int q, int lane) {
  v = wave_sum(v);
  if (lane == 0) red[q * 8 + slot] = v;
  return v;
}

template <typename T, bool FUSED>
__global__ __launch_bounds__(kThreads) void k_adjoint(const AdjArgs<T> D) {
  extern __shared__ __align__(16) unsigned char smem[];
  const AnaArgs<T> &A = D.F;
  const int tid = threadIdx.x;
  const int q = tid >> 6, lane = tid & 63;
  const int c16 = lane & 15, k4 = lane >> 4;
  const int item = A.item_base + (int)blockIdx.x;
  if (item >= A.n_items) return;
  const DomItem it = A.items[item];
  const InstDesc in = A.inst[it.inst];
  const int m = in.m, nown = it.n_own, nobs = it.n_obs, p = 2 * nobs;
  T *xs = (T *)(smem + A.off_xs);
  T *xm = (T *)(smem + A.off_xm);
  double *sg = (double *)(smem + A.off_sg);
  double *dd = (double *)(smem + A.off_dd);
  T *yb = (T *)(smem + A.off_yb);
  int *pn = (int *)(smem + A.off_pn);
  double *sm = (double *)(smem + A.off_s);
  unsigned char *U = smem + A.off_u;
  double *Ub = (double *)U;
  T *Qs = (T *)(smem + D.off_q);  // Q in the state's precision; S after the DK stage
  double *sa = (double *)(smem + D.off_sa);
  const int64_t slot0 = 2 * (int64_t)it.obs_off;

  double X[8], Y[8];
  const CoreStatus st = analysis_core<T, FUSED>(A, it, in, D.frame, smem, X, Y);

  if (st.bad || !st.conv || !st.lam_ok) {
    // the forward kept the forecast on the owned rows: X_a = X' + x_b 1^T
    for (int i = q; i < nown; i += kWaves) {
      const int64_t e = in.x_off + (int64_t)pn[i] * m + lane;
      const double v = lane < m ? (double)D.xbar[e] : 0.0;
      if (lane < m) D.xpbar[e] = (T)v;
      const double s = wave_sum(v);
      if (lane == 0) D.xbbar[in.node_off + pn[i]] = s;
    }
    for (int e = tid; e < p * kLanes; e += kThreads) D.ybar[slot0 * kLanes + e] = (T)0;
    if (tid < p) D.dbar[slot0 + tid] = 0.0;
    if (tid < 4) D.theta[(int64_t)item * 4 + tid] = 0.0;
    return;
  }
  const double kc = (double)(m - 1) / in.rho;

  // ---- A1. Q = U Lambda^{-1/2} into LDS (the state's precision) ----
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int px = pos_x(q, j), py = pos_y(q, j);
    Qs[lane * kQStride + px] = (T)(X[j] / sqrt(sm[S_LAMV + px]));
    Qs[lane * kQStride + py] = (T)(Y[j] / sqrt(sm[S_LAMV + py]));
  }
  // ---- A2. adjoint of the owned rows: read from the global array where used ----
  const T *xab = D.xbar + in.x_off;  // row pn[i], member j at pn[i] * m + j
  if (tid < nown) {
    double s = 0.0;
    for (int j = 0; j < m; ++j) s += (double)xab[(int64_t)pn[tid] * m + j];
    sa[A_XAB + tid] = s;
  }
  __syncthreads();

  // ---- A3. X' W and Xa_bar W on the owned rows (matrix cores, T) ----
  const T *wmat = (const T *)U;
  const double srho = sqrt(in.rho);
  double rho1 = 0.0;
  for (int I = 0; I * 16 < nown; ++I) {
    typename Mfma<T>::V oP = Mfma<T>::zero(), oR = Mfma<T>::zero();
    const int ia = 16 * I + c16;
    const T mu = ia < nown ? xm[ia] : (T)0;
    for (int kk = 0; kk < 16; ++kk) {
      const int k = 4 * kk + k4;
      const bool ok = ia < nown && k < m;
      const T av = ok ? xs[ia * kXsStride + k] - mu : (T)0;
      const T rv = ok ? xab[(int64_t)pn[ia] * m + k] : (T)0;
      const T bv = wmat[k * kYsStride + 16 * q + c16];
      oP = Mfma<T>::mac(av, bv, oP);
      oR = Mfma<T>::mac(rv, bv, oR);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * I + Mfma<T>::row(lane, r), j = 16 * q + c16;
      if (i < nown && j < m) {
        rho1 += (double)xab[(int64_t)pn[i] * m + j] * (double)oP[r];
        const double v = srho * (double)oR[r] + sa[A_XAB + i] * sm[S_WV + j];
        D.xpbar[in.x_off + (int64_t)pn[i] * m + j] = (T)v;
      }
    }
  }
  if (tid < nown) D.xbbar[in.node_off + pn[tid]] = sa[A_XAB + tid];

  // ---- A4. W_bar = sqrt(rho) X'^T Xa_bar (FP64 matrix cores), w_bar ----
  f64x4 wbt[4];
  double kb1 = 0.0;
  {
    const int i = 16 * q + c16;  // row of W_bar = member of X'
#pragma unroll
    for (int J = 0; J < 4; ++J) {
      f64x4 acc = Mfma<double>::zero();
      for (int kk = 0; 4 * kk < nown; ++kk) {
        const int k = 4 * kk + k4;
        const bool ok = k < nown;
        const double av = (ok && i < m) ? (double)(xs[k * kXsStride + i] - xm[k]) : 0.0;
        const double bv = (ok && 16 * J + c16 < m) ? (double)xab[(int64_t)pn[k] * m + 16 * J + c16] : 0.0;
        acc = Mfma<double>::mac(av, bv, acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        acc[r] *= srho;
        const int ii = 16 * q + Mfma<double>::row(lane, r), jj = 16 * J + c16;
        kb1 += acc[r] * (double)wmat[ii * kYsStride + jj];
      }
      wbt[J] = acc;
    }
  }
  if (q == 0) {
    double s = 0.0;
    if (lane < m)
      for (int k = 0; k < nown; ++k) s += (double)(xs[k * kXsStride + lane] - xm[k]) * sa[A_XAB + k];
    sa[A_WBB + lane] = s;
  }
  __syncthreads();  // W (in U) is no longer read
#pragma unroll
  for (int J = 0; J < 4; ++J)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      Ub[(16 * q + Mfma<double>::row(lane, r)) * kQStride + 16 * J + c16] = wbt[J][r];
  // ---- A5. b_bar = Q Lambda^{-1} Q^T w_bar ----
  if (q == 0) {
    double t = 0.0;
    for (int r = 0; r < 64; ++r) t = fma((double)Qs[r * kQStride + lane], sa[A_WBB + r], t);
    sa[A_TV + lane] = t / sm[S_LAMV + lane];
  }
  __syncthreads();
  if (q == 0) {
    double bb = 0.0;
    for (int c = 0; c < 64; ++c) bb = fma((double)Qs[lane * kQStride + c], sa[A_TV + c], bb);
    sa[A_BB + lane] = bb;
  }

  // ---- A6. A_bar of the transform through the eigenpairs (Daleckii-Krein) ----
  // Four products, each held in the waves' registers until every wave has
  // read its operand in Ub and then stored over it: one FP64 work matrix.
  f64x4 t4[4];
  auto store_t4 = [&]() {
    __syncthreads();  // every read of Ub's operand is done
#pragma unroll
    for (int J = 0; J < 4; ++J)
#pragma unroll
      for (int r = 0; r < 4; ++r) Ub[(16 * q + Mfma<double>::row(lane, r)) * kQStride + 16 * J + c16] = t4[J][r];
    __syncthreads();
  };
#pragma unroll
  for (int J = 0; J < 4; ++J)  // P1 = sym(W_bar) Q
    t4[J] = mm64_tile([&](int i, int k) { return 0.5 * (Ub[i * kQStride + k] + Ub[k * kQStride + i]); },
                      [&](int k, int j) { return (double)Qs[k * kQStride + j]; }, q, J, lane);
  store_t4();
  const double skc = sqrt(kc);
#pragma unroll
  for (int J = 0; J < 4; ++J) {  // M = F o (Q^T P1), times sqrt(k)
    t4[J] = mm64_tile([&](int i, int k) { return (double)Qs[k * kQStride + i]; },
                      [&](int k, int j) { return Ub[k * kQStride + j]; }, q, J, lane);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * q + Mfma<double>::row(lane, r), j = 16 * J + c16;
      const double si = sqrt(sm[S_LAMV + i]), sj = sqrt(sm[S_LAMV + j]);
      t4[J][r] *= -skc / (si * sj * (si + sj));
    }
  }
  store_t4();
#pragma unroll
  for (int J = 0; J < 4; ++J)  // P2 = Q M
    t4[J] = mm64_tile([&](int i, int k) { return (double)Qs[i * kQStride + k]; },
                      [&](int k, int j) { return Ub[k * kQStride + j]; }, q, J, lane);
  store_t4();
#pragma unroll
  for (int J = 0; J < 4; ++J)  // P2 Q^T
    t4[J] = mm64_tile([&](int i, int k) { return Ub[i * kQStride + k]; },
                      [&](int k, int j) { return (double)Qs[j * kQStride + k]; }, q, J, lane);
  store_t4();
  // S = sym(A_bar) over Q (no longer read), in the state's precision
  T *Ss = Qs;
  double tr = 0.0;
  for (int e = tid; e < 64 * 64; e += kThreads) {
    const int i = e >> 6, j = e & 63;
    const double v = 0.5 * (Ub[i * kQStride + j] + Ub[j * kQStride + i]) -
                     0.5 * (sa[A_BB + i] * sm[S_WV + j] + sm[S_WV + i] * sa[A_BB + j]);
    Ss[i * kQStride + j] = (T)v;
    if (i == j) tr += v;
  }
  __syncthreads();

  // ---- A7. unscaled local slope anomalies (U), taper derivative, innovation ----
  T *yu = (T *)U;
  for (int o = q; o < nobs; o += kWaves) {
    const uint32_t cw = A.obs_corner[it.obs_off + o];
    const int ca = cw & 255, cb = (cw >> 8) & 255, cc = (cw >> 16) & 255, cd = cw >> 24;
    const T pa = xs[ca * kXsStride + lane], pb = xs[cb * kXsStride + lane];
    const T pc = xs[cc * kXsStride + lane], pd = xs[cd * kXsStride + lane];
    const T sx = (T)0.5 * ((pb - pa) + (pd - pc)) - yb[o];
    const T sy = (T)0.5 * ((pc - pa) + (pd - pb)) - yb[nobs + o];
    yu[o * kYsStride + lane] = lane < m ? sx : (T)0;
    yu[(nobs + o) * kYsStride + lane] = lane < m ? sy : (T)0;
  }
  if (tid < nobs) {
    const int k = A.obs_sub[it.obs_off + tid];
    const double rx = A.r_diag[in.y_off + k], ry = A.r_diag[in.y_off + in.n_subaps + k];
    double dfdc = 0.0;
    if (in.taper_c > 0.0) {
      const double dist = A.obs_dist[it.obs_off + tid];
      const double z = dist / in.taper_c;
      dfdc = -gaspari_cohn_dz(z) * z / in.taper_c;
    }
    sa[A_KAP + tid] = dfdc / sqrt(in.r_scale * rx);
    sa[A_KAP + nobs + tid] = dfdc / sqrt(in.r_scale * ry);
    sa[A_DIN + tid] = (double)A.y[in.y_off + k] - (double)yb[tid];
    sa[A_DIN + nobs + tid] = (double)A.y[in.y_off + in.n_subaps + k] - (double)yb[nobs + tid];
  }
  __syncthreads();

  // ---- A8. Yt_bar = 2 Yt S + dt b_bar^T (FP64 matrix cores), slots ----
  double sacc = 0.0, cacc = 0.0;
  for (int I = 0; 16 * I < p; ++I) {
    f64x4 acc = Mfma<double>::zero();
    const int ia = 16 * I + c16;
    const double sgi = ia < p ? sg[ia] : 0.0;
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
      const int k = 4 * kk + k4;
      const double av = ia < p ? sgi * (double)yu[ia * kYsStride + k] : 0.0;
      acc = Mfma<double>::mac(av, (double)Ss[k * kQStride + 16 * q + c16], acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * I + Mfma<double>::row(lane, r), j = 16 * q + c16;
      if (i < p) {
        double out = 0.0;
        if (j < m) {
          const double yij = (double)yu[i * kYsStride + j];
          const double ytb = 2.0 * acc[r] + dd[i] * sa[A_BB + j];
          sacc += ytb * sg[i] * yij;
          cacc += ytb * yij * sa[A_KAP + i];
          out = sg[i] * ytb;
        }
        D.ybar[(slot0 + i) * kLanes + j] = (T)out;
      }
    }
  }
  // ---- A9. dt_bar = Yt b_bar ----
  if (tid < p) {
    double t = 0.0;
    for (int j = 0; j < m; ++j) t = fma((double)yu[tid * kYsStride + j], sa[A_BB + j], t);
    const double dtb = sg[tid] * t;
    sacc += dtb * dd[tid];
    cacc += dtb * sa[A_DIN + tid] * sa[A_KAP + tid];
    D.dbar[slot0 + tid] = sg[tid] * dtb;
  }
  // ---- A10. (rho, s, c) adjoints of this item ----
  double *red = sa + A_RED;
  block_sum4(rho1, red, 0, q, lane);
  block_sum4(kb1, red, 1, q, lane);
  block_sum4(tr, red, 2, q, lane);
  block_sum4(sacc, red, 3, q, lane);
  block_sum4(cacc, red, 4, q, lane);
  __syncthreads();
  if (tid == 0) {
    double v[5];
    for (int s = 0; s < 5; ++s) v[s] = (red[s] + red[8 + s]) + (red[16 + s] + red[24 + s]);
    const double kbar = v[1] / (2.0 * kc) + v[2];
    double *th = D.theta + (int64_t)item * 4;
    th[0] = v[0] / (2.0 * srho) - kbar * (double)(m - 1) / (in.rho * in.rho);
    th[1] = -v[3] / (2.0 * in.r_scale);
    th[2] = v[4];
    th[3] = 0.0;
  }
}

// Node pass of the frame adjoint (blockIdx.y = instance, one wavefront per
// node, lane = member): the per-slot slope adjoints summed per slope and sent
// through D^T (each node is corner a, b, c or d of up to four subapertures),
// then the anomaly and mean adjoints combined into X_b's and scaled by the AR
// coefficient: the adjoint of the previous analysis ensemble.
template <typename T>
__global__ void k_adjoint_nodes(const InstDesc *insts, const int32_t *node_adj,
                                const int32_t *slot_off, const int32_t *slots, const T *xpbar,
                                const double *xbbar, const T *ybar, const double *dbar, T *xbar_out) {
  const InstDesc in = insts[blockIdx.y];
  const int g = (int)blockIdx.x * kWaves + ((int)threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (g >= in.n_nodes) return;
  const int m = in.m;
  const int64_t gn = in.node_off + g;
  const int64_t e = in.x_off + (int64_t)g * m + lane;
  double acc = lane < m ? (double)xpbar[e] : 0.0;
  double xb = xbbar[gn];
  for (int role = 0; role < 4; ++role) {
    const int sidx = node_adj[4 * gn + role];
    if (sidx < 0) continue;
    const double cx = (role & 1) ? 0.5 : -0.5;
    const double cy = (role & 2) ? 0.5 : -0.5;
    for (int t = slot_off[sidx]; t < slot_off[sidx + 1]; ++t) {
      const int64_t sx = slots[2 * t], sy = sx + slots[2 * t + 1];
      if (lane < m) acc += cx * (double)ybar[sx * kLanes + lane] + cy * (double)ybar[sy * kLanes + lane];
      xb -= cx * dbar[sx] + cy * dbar[sy];
    }
  }
  const double mean = wave_sum(acc) / (double)m;
  if (lane < m) xbar_out[e] = (T)(in.a * (acc - mean + xb / (double)m));
}

// Sum over the threads of a 256-thread block (result in every thread).
// Residual variance of the analysis mean against the true phase:
// stats[2 i] = mean error, stats[2 i + 1] = variance; acc[i] += weights[i] *
// variance when acc is given.  k_resvar_part: kResvarBlocks workgroups per
// instance (blockIdx.y), each a contiguous run of nodes, one wavefront per
// node (lanes over the members); it sums d = e - e_0 and d^2, e the node's
// error and e_0 node 0's (every workgroup forms e_0 alike: the shift keeps
// the one-pass variance clear of cancellation when the mean error is large
// against the spread).  k_resvar_finish adds the partial sums in a fixed
// order.  Deterministic for any launch.
constexpr int kResvarBlocks = 64;

template <typename T>
__device__ inline double node_error(const InstDesc &in, const T *x, const T *truth, int g, int lane) {
  const int m = in.m;
  double v = 0.0;
  for (int k = lane; k < m; k += 64) v += (double)x[in.x_off + (int64_t)g * m + k];
  return wave_sum(v) / (double)m - (double)truth[in.node_off + g];
}

template <typename T>
__global__ __launch_bounds__(256) void k_resvar_part(const InstDesc *insts, const T *x, const T *truth,
                                                    double *part) {
  __shared__ double red[8];
  const InstDesc in = insts[blockIdx.y];
  const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int n = in.n_nodes, per = (n + kResvarBlocks - 1) / kResvarBlocks;
  const int g0 = (int)blockIdx.x * per, g1 = min(n, g0 + per);
  const double e0 = node_error(in, x, truth, 0, lane);
  double s1 = 0.0, s2 = 0.0;
  for (int g = g0 + q; g < g1; g += 4) {
    const double d = node_error(in, x, truth, g, lane) - e0;
    s1 += d;
    s2 = fma(d, d, s2);
  }
  if (lane == 0) {
    red[2 * q] = s1;
    red[2 * q + 1] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* o = part + 2 * ((int64_t)blockIdx.y * kResvarBlocks + blockIdx.x);
    o[0] = (red[0] + red[2]) + (red[4] + red[6]);
    o[1] = (red[1] + red[3]) + (red[5] + red[7]);
  }
}

template <typename T>
__global__ __launch_bounds__(64) void k_resvar_finish(const InstDesc *insts, const T *x, const T *truth,
                                                     const double *part, const double *weights, double *stats,
                                                     double *acc) {
  const InstDesc in = insts[blockIdx.x];
  const int lane = threadIdx.x;
  const double e0 = node_error(in, x, truth, 0, lane);
  const double *pp = part + 2 * (int64_t)blockIdx.x * kResvarBlocks;
  const double s1 = wave_sum(lane < kResvarBlocks ? pp[2 * lane] : 0.0);
  const double s2 = wave_sum(lane < kResvarBlocks ? pp[2 * lane + 1] : 0.0);
  const double n = (double)in.n_nodes, dbar = s1 / n;
  const double var = fma(-dbar, dbar, s2 / n);
  if (lane == 0) {
    stats[2 * blockIdx.x] = e0 + dbar;
    stats[2 * blockIdx.x + 1] = var;
    if (acc) acc[blockIdx.x] += weights[blockIdx.x] * var;
  }
}

// xbar += weights[i] d var / d X_a (blockIdx.y = instance, a wavefront per node).
template <typename T>
__global__ void k_resvar_adjoint(const InstDesc *insts, const T *x, const T *truth,
                                 const double *weights, const double *stats, T *xbar) {
  const InstDesc in = insts[blockIdx.y];
  const int g = (int)blockIdx.x * kWaves + ((int)threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (g >= in.n_nodes) return;
  const int m = in.m;
  const int64_t e = in.x_off + (int64_t)g * m;
  double v = 0.0;
  for (int k = lane; k < m; k += 64) v += (double)x[e + k];
  const double err = wave_sum(v) / (double)m - (double)truth[in.node_off + g] - stats[2 * blockIdx.y];
  const double coef = weights[blockIdx.y] * 2.0 * err / ((double)in.n_nodes * (double)m);
  for (int k = lane; k < m; k += 64) xbar[e + k] = (T)((double)xbar[e + k] + coef);
}

// theta_acc[3 i + t] += sum over the items of instance i of theta[4 item + t]:
// one workgroup per (t, instance), strided partial sums and a fixed-order
// tree (deterministic).
__global__ __launch_bounds__(256) void k_theta_sum(const int32_t *dom_base, const double *theta,
                                                  double *theta_acc) {
  __shared__ double red[4];
  const int t = blockIdx.x, inst = blockIdx.y;
  const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double s = 0.0;
  for (int k = dom_base[inst] + (int)threadIdx.x; k < dom_base[inst + 1]; k += 256) s += theta[4 * (int64_t)k + t];
  s = wave_sum(s);
  if (lane == 0) red[q] = s;
  __syncthreads();
  if (threadIdx.x == 0) theta_acc[3 * inst + t] += (red[0] + red[1]) + (red[2] + red[3]);
}

// ------------------------------------------------- differential pistons
// Least-squares removal of one piston per domain after the gather (Sec.
// 4.4): pi = M^+ P^T D^T (y - D x_a) with P the node-to-domain indicator and
// M = P^T D^T D P (only subapertures with corners in two or more domains
// contribute); M^+ is precomputed per instance.  Then every member of a node
// gets the piston of its domain.  One wavefront per domain or node.
template <typename T> struct PistonArgs {
  const InstDesc *inst;
  const DomItem *items;
  int32_t n_items, pad0;
  const int32_t *patch_node;   // owned nodes first
  const int32_t *node_adj;     // per global node: subaperture of corner role a, b, c, d (-1)
  const int32_t *subap_nodes;  // per global subaperture: its 4 corner nodes (instance-local)
  const int32_t *owner_item;   // per global node: the work item owning it
  const int32_t *dom_base;     // first item of each instance (+ total)
  const int64_t *minv_off;     // offset of each instance's M^+ (nd x nd, row-major)
  const double *minv;
  const T *x_mean;             // analysis mean per global node
  const T *y;                  // slopes
  double *rhs;                 // per item (forward: P^T D^T residual; adjoint: P^T Z_bar 1)
  double *pi;                  // per item (forward: pistons; adjoint: M^+ of the sums)
  T *x;                        // ensemble updated in place
  const int32_t *term_off;     // per item: its right-hand-side terms (+ total); NULL: 64 a item
  const PistonTerm *terms;
  const PistonItem *pitem;     // per item: what the piston step reads
};

// rhs[item] = sum over the owned nodes of (D^T (y - D x_mean))_node: only
// the subapertures the domain shares with others contribute (the corners'
// coefficients of a subaperture inside one domain sum to zero), each with
// the summed coefficients of the domain's own corners, from a table built at
// create: at a fixed stride of 64 an item when every item has at most 64
// (one load before the means and slopes; unused entries have coefficients
// 0 and node 0), else through per-item offsets.
template <typename T> __global__ void k_piston_rhs(const PistonArgs<T> P) {
  const int item = (int)blockIdx.x * kWaves + ((int)threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (item >= P.n_items) return;
  int t0, t1, st;
  if (P.term_off) {
    t0 = P.term_off[item];
    t1 = P.term_off[item + 1];
    st = 64;
  } else {
    t0 = 64 * item;
    t1 = t0 + 64;
    st = 64;
  }
  double v = 0.0;
  for (int t = t0 + lane; t < t1; t += st) {
    const PistonTerm pt = P.terms[t];
    const double xa = (double)P.x_mean[pt.c[0]], xb = (double)P.x_mean[pt.c[1]];
    const double xc = (double)P.x_mean[pt.c[2]], xd = (double)P.x_mean[pt.c[3]];
    const double ex = (double)P.y[pt.yx] - 0.5 * ((xb - xa) + (xd - xc));
    const double ey = (double)P.y[pt.yy] - 0.5 * ((xc - xa) + (xd - xb));
    // (an unused entry adds nothing, also where its slopes are not finite)
    if (pt.cx != 0.0f || pt.cy != 0.0f) v = fma((double)pt.cx, ex, fma((double)pt.cy, ey, v));
  }
  v = wave_sum(v);
  if (lane == 0) P.rhs[item] = v;
}

// pi[item] = row of M^+ times rhs over the items of the same instance.
template <typename T> __global__ void k_piston_solve(const PistonArgs<T> P) {
  const int item = (int)blockIdx.x * kWaves + ((int)threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (item >= P.n_items) return;
  const int inst = P.items[item].inst;
  if (!P.inst[inst].piston) {
    if (lane == 0) P.pi[item] = 0.0;
    return;
  }
  const int b0 = P.dom_base[inst], nd = P.dom_base[inst + 1] - b0;
  const double *row = P.minv + P.minv_off[inst] + (int64_t)(item - b0) * nd;
  double v = 0.0;
  for (int e = lane; e < nd; e += 64) v = fma(row[e], P.rhs[b0 + e], v);
  v = wave_sum(v);
  if (lane == 0) P.pi[item] = v;
}

// x[node][j] += pi[owner(node)] (blockIdx.y = instance).
template <typename T> __global__ void k_piston_apply(const PistonArgs<T> P) {
  const InstDesc in = P.inst[blockIdx.y];
  if (!in.piston) return;
  const int64_t n = (int64_t)in.n_nodes * in.m;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t node = e / in.m;
    const double pv = P.pi[P.owner_item[in.node_off + node]];
    P.x[in.x_off + e] = (T)((double)P.x[in.x_off + e] + pv);
  }
}

// pi of each domain (a row of M^+ times rhs) added to every member of its
// owned nodes: one workgroup per item, the row's products spread over the
// workgroup (a few loads a thread, all in flight at once) while the owned rows
// load.  Item 0 also advances the frame counter of the bank draws when
// `frame` is given (the last step of the frame).
template <typename T> __global__ void k_piston_finish(const PistonArgs<T> P, uint32_t *frame) {
  __shared__ double pi_w[kWaves];
  const int item = blockIdx.x;
  const int tid = threadIdx.x, q = tid >> 6, lane = tid & 63;
  if (frame && item == 0 && tid == 0) *frame += 1u;
  const PistonItem pr = P.pitem[item];  // one load before the row and the owned rows
  if (!pr.piston) return;
  // the owned rows are loaded (eight elements a thread a pass) while the
  // workgroup forms the piston
  const int m = pr.m, ne = pr.n_own * m;
  double pv = 0.0;
  for (int e0 = 0; e0 < ne; e0 += 8 * kThreads) {
    T xv[8];
    int64_t xi[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * kThreads + tid, ec = e < ne ? e : 0;
      const int i = ec / m, j = ec - i * m;
      xi[u] = pr.x_off + (int64_t)P.patch_node[pr.patch_off + i] * m + j;
      xv[u] = P.x[xi[u]];
    }
    if (e0 == 0) {
      const double *row = P.minv + pr.row;
      double v = 0.0;
      for (int e = tid; e < pr.nd; e += kThreads) v = fma(row[e], P.rhs[pr.b0 + e], v);
      v = wave_sum(v);
      if (lane == 0) pi_w[q] = v;
      __syncthreads();
      pv = sum4(pi_w);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (e0 + u * kThreads + tid < ne) P.x[xi[u]] = (T)((double)xv[u] + pv);
  }
}

// The command of the closed loop (Sec. 2.2 control part): u_k = P phi^_{k+1/k}
// with a zonal DM (N = P = I) and the two-step prediction of the analysed
// phase phi_{k-1}: u_k = a^2 x_a.  The history moves on: u_{k-2} <- u_{k-1},
// u_{k-1} <- u_k.  One wavefront per node (lane = member), grid (nodes / 4,
// instances); instances of the delay-free model are left alone.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_command(const InstDesc *insts, const T *x, T *u1, T *u2) {
  const InstDesc in = insts[blockIdx.y];
  const int g = (int)blockIdx.x * kWaves + ((int)threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (in.model != 1 || g >= in.n_nodes) return;
  const int m = in.m;
  const double v = lane < m ? (double)x[in.x_off + (int64_t)g * m + lane] : 0.0;
  const double mean = wave_sum(v) / m;
  if (lane == 0) {
    const int64_t e = in.node_off + g;
    u2[e] = u1[e];
    u1[e] = (T)(in.a * in.a * mean);
  }
}

// Adjoint: rhs[item] = sum over the owned nodes and members of Z_bar.
template <typename T> __global__ void k_piston_adj_sum(const PistonArgs<T> P) {
  const int item = (int)blockIdx.x * kWaves + ((int)threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (item >= P.n_items) return;
  const DomItem it = P.items[item];
  const InstDesc in = P.inst[it.inst];
  double v = 0.0;
  if (in.piston && lane < in.m)
    for (int i = 0; i < it.n_own; ++i)
      v += (double)P.x[in.x_off + (int64_t)P.patch_node[it.patch_off + i] * in.m + lane];
  v = wave_sum(v);
  if (lane == 0) P.rhs[item] = v;
}

// Adjoint: x[node][j] -= (D^T D P t)_node / m with t = pi (blockIdx.y =
// instance, one wavefront per node).
template <typename T> __global__ void k_piston_adj_apply(const PistonArgs<T> P) {
  const InstDesc in = P.inst[blockIdx.y];
  if (!in.piston) return;
  const int g = (int)blockIdx.x * kWaves + ((int)threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (g >= in.n_nodes) return;
  const int64_t gn = in.node_off + g;
  double v = 0.0;
  for (int role = 0; role < 4; ++role) {
    const int s = P.node_adj[4 * gn + role];
    if (s < 0) continue;
    const int32_t *c = P.subap_nodes + 4 * (int64_t)s;
    const double ta = P.pi[P.owner_item[in.node_off + c[0]]], tb = P.pi[P.owner_item[in.node_off + c[1]]];
    const double tc = P.pi[P.owner_item[in.node_off + c[2]]], td = P.pi[P.owner_item[in.node_off + c[3]]];
    const double rx = 0.5 * ((tb - ta) + (td - tc));
    const double ry = 0.5 * ((tc - ta) + (td - tb));
    v += ((role & 1) ? 0.5 : -0.5) * rx + ((role & 2) ? 0.5 : -0.5) * ry;
  }
  if (lane < in.m) {
    const int64_t e = in.x_off + (int64_t)g * in.m + lane;
    P.x[e] = (T)((double)P.x[e] - v / (double)in.m);
  }
}

// Forecast X_b = a X_a + V over every instance (blockIdx.y = instance).
template <typename T>
__global__ void k_forecast(const InstDesc *insts, const int32_t *node_ij, const T *xa, const T *v,
                           const float *bank, const uint32_t *frame, T *xb, const T *xprev) {
  const InstDesc in = insts[blockIdx.y];
  const int64_t n = (int64_t)in.n_nodes * in.m;
  const T a = (T)in.a;
  const T a2 = (T)in.a2;
  const bool use_prev = xprev && in.a2 != 0.0;
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
    noise *= (T)in.vscale;
    if (use_prev) noise = fma_t(a2, xprev[in.x_off + e], noise);
    xb[in.x_off + e] = fma_t(a, xa[in.x_off + e], noise);
  }
}

// dst <- src over n elements (the AR(2) history, kept as a kernel so that it
// can sit in the frame graph).
template <typename T> __global__ void k_copy(const T *src, T *dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

// Online refit of the AR(1) model (Sec. 4.2: the model may be re-identified
// while the filter runs).  Per instance and frame, the lag-1 pair of analysis
// means x_k = mean of X_a(k), x_{k-1} = mean of X_a(k-1) gives four sums over
// the nodes: <x_k>, <x_{k-1}>, x_k . x_{k-1}, x_{k-1} . x_{k-1}.  One
// wavefront per node (lane = member), grid (ceil(max nodes / 4), instances);
// each workgroup writes its four partial sums to part[(inst * stride + block) * 4].
template <typename T>
__global__ __launch_bounds__(kThreads) void k_refit_sums(const InstDesc *insts, const RefitState *rs,
                                                         const T *x_now, const T *x_prev, double *part,
                                                         int stride) {
  const int inst = blockIdx.y;
  const InstDesc in = insts[inst];
  if (rs[inst].f == 0.0 || (int)blockIdx.x * kWaves >= in.n_nodes) return;  // whole workgroup
  __shared__ double red[kWaves][4];
  const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = (int)blockIdx.x * kWaves + q, m = in.m;
  double xn = 0.0, xp = 0.0;
  if (g < in.n_nodes && lane < m) {
    const int64_t e = in.x_off + (int64_t)g * m + lane;
    xn = (double)x_now[e];
    xp = (double)x_prev[e];
  }
  xn = wave_sum(xn) / m;
  xp = wave_sum(xp) / m;
  if (lane == 0) {
    const bool v = g < in.n_nodes;
    red[q][0] = v ? xn : 0.0;
    red[q][1] = v ? xp : 0.0;
    red[q][2] = v ? xn * xp : 0.0;
    red[q][3] = v ? xp * xp : 0.0;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double t = 0.0;
    for (int w = 0; w < kWaves; ++w) t += red[w][threadIdx.x];
    part[((int64_t)inst * stride + blockIdx.x) * 4 + threadIdx.x] = t;
  }
}

// The refit's update, one workgroup per instance: the partial sums reduced in
// a fixed order, the piston-removed products
//   c01 = x_k . x_{k-1} - n <x_k> <x_{k-1}>,   c11 = |x_{k-1}|^2 - n <x_{k-1}>^2,
// folded in with forgetting f (s01 = f s01 + c01, s11 = f s11 + c11), and the
// model of the next frames: a = clip(s01 / s11, 0, a_max) once s11 > 0, and
// the factor on the model noise (drawn for a_0) that keeps the stationary
// variance, sqrt((1 - a^2) / (1 - a_0^2)).
__global__ __launch_bounds__(kThreads) void k_refit_finish(InstDesc *insts, RefitState *rs,
                                                           const double *part, int stride) {
  const int inst = blockIdx.x;
  if (rs[inst].f == 0.0) return;
  const int n = insts[inst].n_nodes, nb = (n + kWaves - 1) / kWaves;
  __shared__ double red[kWaves][4];
  const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += kThreads) {
    const double *p = part + ((int64_t)inst * stride + b) * 4;
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] += p[c];
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double v = wave_sum(acc[c]);
    if (lane == 0) red[q][c] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double S[4];
    for (int c = 0; c < 4; ++c) {
      S[c] = 0.0;
      for (int w = 0; w < kWaves; ++w) S[c] += red[w][c];
    }
    RefitState r = rs[inst];
    const double c01 = S[2] - S[0] * S[1] / n, c11 = S[3] - S[1] * S[1] / n;
    r.s01 = r.f * r.s01 + c01;
    r.s11 = r.f * r.s11 + c11;
    r.frames += 1;
    rs[inst] = r;
    if (r.s11 > 0.0) {
      const double a = fmin(fmax(r.s01 / r.s11, 0.0), r.a_max);
      insts[inst].a = a;
      insts[inst].vscale = sqrt((1.0 - a * a) / (1.0 - r.a0 * r.a0));
    }
  }
}

// Blend-mode gather (a variant of the Sec. 4.2 concatenation): every domain
// has analysed all rows of its node patch into `stage` ([patch entry][64])
// and their member means into `smean`.  The patches are first put on a
// common piston: pi minimises the squared differences of the means of every
// node held by two patches, i.e. L pi = rhs with L the graph Laplacian
// weighted by the number of shared nodes (geometry only: its pseudo-inverse
// is built once) and rhs_l = sum over the rows of patch l of the summed
// differences (other patch's mean - this patch's mean) at that node.  Then
// every node takes the normalised tent-weighted mean of its patch rows plus
// their pistons.  The node -> (entry, item, weight) lists are in item order,
// so every sum runs in a fixed order.

// rhs[item], one wavefront per item (lane = patch row).
__global__ __launch_bounds__(kThreads) void k_blend_rhs(const InstDesc *insts, const DomItem *items, int n_items,
                                                        const int32_t *patch_node, const double *smean,
                                                        const int32_t *boff, const int32_t *bent, double *rhs) {
  const int item = (int)blockIdx.x * kWaves + ((int)threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (item >= n_items) return;  // whole wavefront
  const DomItem it = items[item];
  const InstDesc in = insts[it.inst];
  if (!in.blend) return;
  double v = 0.0;
  if (lane < it.n_patch) {
    const int e0 = it.patch_off + lane;
    const int64_t node = in.node_off + patch_node[e0];
    const double self = smean[e0];
    for (int k = boff[node]; k < boff[node + 1]; ++k) v += smean[bent[k]] - self;
  }
  v = wave_sum(v);
  if (lane == 0) rhs[item] = v;
}

// pi[item] = row of L^+ times the instance's rhs, one wavefront per item.
__global__ __launch_bounds__(kThreads) void k_blend_solve(const InstDesc *insts, const DomItem *items, int n_items,
                                                          const int32_t *dom_base, const int64_t *minv_off,
                                                          const double *minv, const double *rhs, double *pi) {
  const int item = (int)blockIdx.x * kWaves + ((int)threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (item >= n_items) return;  // whole wavefront
  const DomItem it = items[item];
  if (!insts[it.inst].blend) return;
  const int b0 = dom_base[it.inst], nd = dom_base[it.inst + 1] - b0;
  const double *row = minv + minv_off[it.inst] + (int64_t)(item - b0) * nd;
  double v = 0.0;
  for (int e = lane; e < nd; e += 64) v = fma(row[e], rhs[b0 + e], v);
  v = wave_sum(v);
  if (lane == 0) pi[item] = v;
}

// X_a(node) = sum_k w_k (stage row k + pi of its item), one wavefront per node
// (lane = member), grid (ceil(max nodes / 4), instances); the frame counter
// of the bank draws advances here when `frame` is given.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_blend_gather(const InstDesc *insts, const int32_t *boff,
                                                           const int32_t *bent, const int32_t *bitem,
                                                           const double *bw, const T *stage, const double *pi,
                                                           T *x, uint32_t *frame) {
  if (frame && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *frame += 1u;
  const InstDesc in = insts[blockIdx.y];
  const int g = (int)blockIdx.x * kWaves + ((int)threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (!in.blend || g >= in.n_nodes || lane >= in.m) return;
  const int64_t node = in.node_off + g;
  double acc = 0.0;
  for (int k = boff[node]; k < boff[node + 1]; ++k)
    acc = fma(bw[k], (double)stage[(int64_t)bent[k] * 64 + lane] + pi[bitem[k]], acc);
  x[in.x_off + (int64_t)g * in.m + lane] = (T)acc;
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

// Stand-alone SPD eigensolve with the same distributed Cholesky + Jacobi,
// one workgroup per matrix.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_eigh_spd(const double *Am, int m, double tol,
                                                       int max_sweeps, double *Q, double *lam_out,
                                                       int32_t *sweeps_out) {
  __shared__ double smem_s[S_TOTAL];
  __shared__ double la_s[64 * kLaStride];  // the matrix, then the exchange area
  const int tid = threadIdx.x, q = tid >> 6, r = tid & 63;
  const double *Ab = Am + (int64_t)blockIdx.x * m * m;
  for (int e = tid; e < 64 * 64; e += kThreads) {
    const int i = e >> 6, j = e & 63;
    la_s[i * kLaStride + j] = (i < m && j < m) ? Ab[i * m + j] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  double X[8], Y[8];
  double *sm = smem_s;
  cholesky_lds(la_s, sm, q, r);
  load_dist(la_s, X, Y, q, r);
  __syncthreads();
  const int sw = jacobi_dist(X, Y, sm, la_s, tol, max_sweeps, true, q, r);  // columns < m are A's
  column_sums(X, Y, [](double v) { return v * v; }, sm + S_LAM, q, r);
  __syncthreads();
  if (r < m) {
    double *Qb = Q + (int64_t)blockIdx.x * m * m;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int px = pos_x(q, j), py = pos_y(q, j);
      if (px < m) Qb[r * m + px] = X[j] / sqrt(sm[S_LAM + px]);
      if (py < m) Qb[r * m + py] = Y[j] / sqrt(sm[S_LAM + py]);
    }
    if (q == 0) lam_out[(int64_t)blockIdx.x * m + r] = sm[S_LAM + r];
  }
  if (tid == 0 && sweeps_out) sweeps_out[blockIdx.x] = sw;
}

}  // namespace letkf

// ---------------------------------------------------------------------------
// Fixed device scratch of letkf_adjoint_noalloc: the per-call buffers of the
// adjoint (node and slope adjoint slots, per-item partials) for callers that
// cannot allocate.  Each device holds its own copy for the life of the
// process; host code reaches it only through the address that
// hipGetSymbolAddress gives on that device.
constexpr size_t kNoallocScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

extern "C" size_t letkf_noalloc_scratch_bytes(void) { return kNoallocScratchBytes; }

// The device address of `scratch` on the current device (looked up once per
// device, under a lock).  Returns the HIP error of the lookup.
#include <mutex>
extern "C" hipError_t letkf_noalloc_scratch(int device, void **ptr) {
  static std::mutex mu;
  static void *addr[64] = {nullptr};
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = p;
  }
  *ptr = addr[device];
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Launch wrappers called by the host side.
using namespace letkf;

extern "C" const void *letkf_wide_kernel(int fp64, int fused, int nb);
extern "C" int letkf_wide_threads(void);

template <typename T> static const void *analysis_kernel_of(int fused, int eig) {
  if (eig >= kAnalysisWide) return letkf_wide_kernel(sizeof(T) == 8, fused, eig - kAnalysisWide);
  if (eig == kEigCl)
    return fused ? (const void *)k_analysis_cl<T, true> : (const void *)k_analysis_cl<T, false>;
  if (eig == kEigJacobi)
    return fused ? (const void *)k_analysis<T, true, kEigJacobi> : (const void *)k_analysis<T, false, kEigJacobi>;
  if (eig == kEigNs32 && sizeof(T) == 4)
    return fused ? (const void *)k_analysis<T, true, kEigNs32> : (const void *)k_analysis<T, false, kEigNs32>;
  if (eig == kEigNspMix && sizeof(T) == 4)
    return fused ? (const void *)k_analysis<T, true, kEigNspMix> : (const void *)k_analysis<T, false, kEigNspMix>;
  if (eig == kEigNsp || eig == kEigNspMix)
    return fused ? (const void *)k_analysis<T, true, kEigNsp> : (const void *)k_analysis<T, false, kEigNsp>;
  return fused ? (const void *)k_analysis<T, true, kEigNs64> : (const void *)k_analysis<T, false, kEigNs64>;
}

extern "C" const void *letkf_analysis_kernel(int fp64, int fused, int eig) {
  return fp64 ? analysis_kernel_of<double>(fused, eig) : analysis_kernel_of<float>(fused, eig);
}

extern "C" hipError_t letkf_launch_analysis(const void *args, int fp64, int fused, int eig, int grid,
                                            size_t lds, hipStream_t s) {
  void *kargs[] = {(void *)args};
  const void *k = letkf_analysis_kernel(fp64, fused, eig);
  if (!k) return hipErrorInvalidValue;
  return hipLaunchKernel(k, dim3(grid), dim3(eig >= kAnalysisWide ? letkf_wide_threads() : kThreads), kargs, lds, s);
}

// Threads per workgroup of the analysis kernel `eig`.
extern "C" int letkf_analysis_threads_for(int eig) { return eig >= kAnalysisWide ? letkf_wide_threads() : kThreads; }

extern "C" const void *letkf_command_kernel(int fp64) {
  return fp64 ? (const void *)k_command<double> : (const void *)k_command<float>;
}

extern "C" hipError_t letkf_launch_command(int fp64, const InstDesc *insts, int n_inst, int max_nodes,
                                           const void *x, void *u1, void *u2, hipStream_t s) {
  const dim3 grid((max_nodes + kWaves - 1) / kWaves, n_inst);
  if (fp64)
    hipLaunchKernelGGL(k_command<double>, grid, dim3(kThreads), 0, s, insts, (const double *)x,
                       (double *)u1, (double *)u2);
  else
    hipLaunchKernelGGL(k_command<float>, grid, dim3(kThreads), 0, s, insts, (const float *)x,
                       (float *)u1, (float *)u2);
  return hipGetLastError();
}

extern "C" int letkf_analysis_threads(void) { return kThreads; }

extern "C" size_t letkf_analysis_scratch_doubles(void) { return S_TOTAL; }
extern "C" size_t letkf_analysis_fwd_scratch_doubles(void) { return kFwdScratch; }

extern "C" size_t letkf_analysis_xch_bytes(void) {
  return (size_t)kXchBytes;
}

extern "C" const void *letkf_refit_sums_kernel(int fp64) {
  return fp64 ? (const void *)k_refit_sums<double> : (const void *)k_refit_sums<float>;
}

extern "C" const void *letkf_refit_finish_kernel(void) { return (const void *)k_refit_finish; }

// Partial-sum rows per instance of the refit (grid x of k_refit_sums).
extern "C" int letkf_refit_stride(int max_nodes) { return (max_nodes + kWaves - 1) / kWaves; }

extern "C" hipError_t letkf_launch_refit(int fp64, void *insts, void *rs, const void *x_now, const void *x_prev,
                                         double *part, int max_nodes, int n_inst, hipStream_t s) {
  const int stride = letkf_refit_stride(max_nodes);
  const dim3 g(stride, n_inst);
  if (fp64)
    hipLaunchKernelGGL(k_refit_sums<double>, g, dim3(kThreads), 0, s, (const InstDesc *)insts,
                       (const RefitState *)rs, (const double *)x_now, (const double *)x_prev, part, stride);
  else
    hipLaunchKernelGGL(k_refit_sums<float>, g, dim3(kThreads), 0, s, (const InstDesc *)insts,
                       (const RefitState *)rs, (const float *)x_now, (const float *)x_prev, part, stride);
  hipLaunchKernelGGL(k_refit_finish, dim3(n_inst), dim3(kThreads), 0, s, (InstDesc *)insts, (RefitState *)rs,
                     (const double *)part, stride);
  return hipGetLastError();
}

extern "C" const void *letkf_blend_rhs_kernel(void) { return (const void *)k_blend_rhs; }
extern "C" const void *letkf_blend_solve_kernel(void) { return (const void *)k_blend_solve; }
extern "C" const void *letkf_blend_gather_kernel(int fp64) {
  return fp64 ? (const void *)k_blend_gather<double> : (const void *)k_blend_gather<float>;
}

extern "C" hipError_t letkf_launch_blend(int fp64, const InstDesc *insts, const DomItem *items, int n_items,
                                         const int32_t *patch_node, const double *smean, const int32_t *boff,
                                         const int32_t *bent, const int32_t *bitem, const double *bw,
                                         const int32_t *dom_base, const int64_t *minv_off, const double *minv,
                                         double *rhs, double *pi, const void *stage, void *x, uint32_t *frame,
                                         int max_nodes, int n_inst, hipStream_t s) {
  const dim3 gi((n_items + kWaves - 1) / kWaves), gn((max_nodes + kWaves - 1) / kWaves, n_inst);
  hipLaunchKernelGGL(k_blend_rhs, gi, dim3(kThreads), 0, s, insts, items, n_items, patch_node, smean, boff, bent,
                     rhs);
  hipLaunchKernelGGL(k_blend_solve, gi, dim3(kThreads), 0, s, insts, items, n_items, dom_base, minv_off, minv,
                     (const double *)rhs, pi);
  if (fp64)
    hipLaunchKernelGGL(k_blend_gather<double>, gn, dim3(kThreads), 0, s, insts, boff, bent, bitem, bw,
                       (const double *)stage, (const double *)pi, (double *)x, frame);
  else
    hipLaunchKernelGGL(k_blend_gather<float>, gn, dim3(kThreads), 0, s, insts, boff, bent, bitem, bw,
                       (const float *)stage, (const double *)pi, (float *)x, frame);
  return hipGetLastError();
}

extern "C" const void *letkf_copy_kernel(int fp64) {
  return fp64 ? (const void *)k_copy<double> : (const void *)k_copy<float>;
}

extern "C" hipError_t letkf_launch_copy(int fp64, const void *src, void *dst, int64_t n, hipStream_t s) {
  int gx = (int)((n + 255) / 256);
  if (gx > 4096) gx = 4096;
  if (gx < 1) gx = 1;
  if (fp64)
    hipLaunchKernelGGL(k_copy<double>, dim3(gx), dim3(256), 0, s, (const double *)src, (double *)dst, n);
  else
    hipLaunchKernelGGL(k_copy<float>, dim3(gx), dim3(256), 0, s, (const float *)src, (float *)dst, n);
  return hipGetLastError();
}

extern "C" hipError_t letkf_launch_forecast(int fp64, const InstDesc *insts, int n_inst,
                                            const int32_t *node_ij, const void *xa, const void *v,
                                            const float *bank, const uint32_t *frame, void *xb,
                                            const void *xprev, int64_t max_elems, hipStream_t s) {
  int gx = (int)((max_elems + 255) / 256);
  if (gx > 4096) gx = 4096;
  if (gx < 1) gx = 1;
  if (fp64)
    hipLaunchKernelGGL(k_forecast<double>, dim3(gx, n_inst), dim3(256), 0, s, insts, node_ij,
                       (const double *)xa, (const double *)v, bank, frame, (double *)xb,
                       (const double *)xprev);
  else
    hipLaunchKernelGGL(k_forecast<float>, dim3(gx, n_inst), dim3(256), 0, s, insts, node_ij,
                       (const float *)xa, (const float *)v, bank, frame, (float *)xb,
                       (const float *)xprev);
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
  hipLaunchKernelGGL(k_eigh_spd, dim3(batch), dim3(kThreads), 0, s, A, m, tol, max_sweeps, Q, lam,
                     sweeps);
  return hipGetLastError();
}

extern "C" size_t letkf_args_size(int fp64) {
  return fp64 ? sizeof(AnaArgs<double>) : sizeof(AnaArgs<float>);
}

extern "C" const void *letkf_adjoint_kernel(int fp64) {
  return fp64 ? (const void *)k_adjoint<double, true> : (const void *)k_adjoint<float, true>;
}

extern "C" size_t letkf_adjoint_scratch_doubles(void) { return A_TOTAL; }

extern "C" hipError_t letkf_launch_adjoint(int fp64, const void *args, int grid, size_t lds,
                                           hipStream_t s) {
  if (fp64)
    hipLaunchKernelGGL((k_adjoint<double, true>), dim3(grid), dim3(kThreads), lds, s,
                       *(const AdjArgs<double> *)args);
  else
    hipLaunchKernelGGL((k_adjoint<float, true>), dim3(grid), dim3(kThreads), lds, s,
                       *(const AdjArgs<float> *)args);
  return hipGetLastError();
}

extern "C" size_t letkf_adjoint_args_size(int fp64) {
  return fp64 ? sizeof(AdjArgs<double>) : sizeof(AdjArgs<float>);
}

extern "C" hipError_t letkf_launch_adjoint_nodes(int fp64, const InstDesc *insts, int n_inst,
                                                 const int32_t *node_adj, const int32_t *slot_off,
                                                 const int32_t *slots, const void *xpbar,
                                                 const double *xbbar, const void *ybar,
                                                 const double *dbar, void *xbar_out, int max_nodes,
                                                 hipStream_t s) {
  const int gx = (max_nodes + kWaves - 1) / kWaves;
  if (fp64)
    hipLaunchKernelGGL(k_adjoint_nodes<double>, dim3(gx, n_inst), dim3(kThreads), 0, s, insts,
                       node_adj, slot_off, slots, (const double *)xpbar, xbbar,
                       (const double *)ybar, dbar, (double *)xbar_out);
  else
    hipLaunchKernelGGL(k_adjoint_nodes<float>, dim3(gx, n_inst), dim3(kThreads), 0, s, insts,
                       node_adj, slot_off, slots, (const float *)xpbar, xbbar, (const float *)ybar,
                       dbar, (float *)xbar_out);
  return hipGetLastError();
}

// Doubles of the stats buffer letkf_launch_resvar needs for n_inst instances.
extern "C" size_t letkf_resvar_stats_doubles(int n_inst) { return (size_t)2 * n_inst * (1 + kResvarBlocks); }

extern "C" hipError_t letkf_launch_resvar(int fp64, const InstDesc *insts, int n_inst, const void *x,
                                          const void *truth, const double *weights, double *stats,
                                          double *acc, hipStream_t s) {
  // stats holds 2 n_inst results, then the 2 kResvarBlocks n_inst partial sums
  double *part = stats + 2 * n_inst;
  if (fp64) {
    hipLaunchKernelGGL(k_resvar_part<double>, dim3(kResvarBlocks, n_inst), dim3(256), 0, s, insts,
                       (const double *)x, (const double *)truth, part);
    hipLaunchKernelGGL(k_resvar_finish<double>, dim3(n_inst), dim3(64), 0, s, insts, (const double *)x,
                       (const double *)truth, part, weights, stats, acc);
  } else {
    hipLaunchKernelGGL(k_resvar_part<float>, dim3(kResvarBlocks, n_inst), dim3(256), 0, s, insts,
                       (const float *)x, (const float *)truth, part);
    hipLaunchKernelGGL(k_resvar_finish<float>, dim3(n_inst), dim3(64), 0, s, insts, (const float *)x,
                       (const float *)truth, part, weights, stats, acc);
  }
  return hipGetLastError();
}

extern "C" hipError_t letkf_launch_resvar_adjoint(int fp64, const InstDesc *insts, int n_inst,
                                                  const void *x, const void *truth,
                                                  const double *weights, const double *stats,
                                                  void *xbar, int max_nodes, hipStream_t s) {
  const int gx = (max_nodes + kWaves - 1) / kWaves;
  if (fp64)
    hipLaunchKernelGGL(k_resvar_adjoint<double>, dim3(gx, n_inst), dim3(kThreads), 0, s, insts,
                       (const double *)x, (const double *)truth, weights, stats, (double *)xbar);
  else
    hipLaunchKernelGGL(k_resvar_adjoint<float>, dim3(gx, n_inst), dim3(kThreads), 0, s, insts,
                       (const float *)x, (const float *)truth, weights, stats, (float *)xbar);
  return hipGetLastError();
}

extern "C" hipError_t letkf_launch_theta_sum(const int32_t *dom_base, int n_inst, const double *theta,
                                             double *theta_acc, hipStream_t s) {
  hipLaunchKernelGGL(k_theta_sum, dim3(3, n_inst), dim3(256), 0, s, dom_base, theta, theta_acc);
  return hipGetLastError();
}

// Differential pistons: which = 0 rhs, 1 solve, 2 apply, 3 adjoint sums,
// 4 adjoint apply; the kernel and its launch shape for graph nodes too.
extern "C" const void *letkf_piston_kernel(int fp64, int which) {
  if (fp64) {
    const void *k[5] = {(const void *)k_piston_rhs<double>, (const void *)k_piston_solve<double>,
                        (const void *)k_piston_apply<double>, (const void *)k_piston_adj_sum<double>,
                        (const void *)k_piston_adj_apply<double>};
    return k[which];
  }
  const void *k[5] = {(const void *)k_piston_rhs<float>, (const void *)k_piston_solve<float>,
                      (const void *)k_piston_apply<float>, (const void *)k_piston_adj_sum<float>,
                      (const void *)k_piston_adj_apply<float>};
  return k[which];
}

extern "C" const void *letkf_piston_finish_kernel(int fp64) {
  return fp64 ? (const void *)k_piston_finish<double> : (const void *)k_piston_finish<float>;
}

extern "C" hipError_t letkf_launch_piston_finish(int fp64, const void *args, int n_items,
                                                 uint32_t *frame, hipStream_t s) {
  void *kargs[] = {(void *)args, (void *)&frame};
  return hipLaunchKernel(letkf_piston_finish_kernel(fp64), dim3(n_items), dim3(kThreads), kargs, 0, s);
}

extern "C" size_t letkf_piston_args_size(int fp64) {
  return fp64 ? sizeof(PistonArgs<double>) : sizeof(PistonArgs<float>);
}

// Grid of piston kernel `which` (block = kThreads).
extern "C" void letkf_piston_grid(int which, int n_items, int n_inst, int max_nodes,
                                  int64_t max_elems, int *gx, int *gy) {
  if (which == 0 || which == 1 || which == 3) {
    *gx = (n_items + kWaves - 1) / kWaves;
    *gy = 1;
  } else if (which == 2) {
    int64_t b = (max_elems + kThreads - 1) / kThreads;
    *gx = (int)(b < 2048 ? (b < 1 ? 1 : b) : 2048);
    *gy = n_inst;
  } else {
    *gx = (max_nodes + kWaves - 1) / kWaves;
    *gy = n_inst;
  }
}

extern "C" hipError_t letkf_launch_piston(int fp64, int which, const void *args, int gx, int gy,
                                          hipStream_t s) {
  void *kargs[] = {(void *)args};
  return hipLaunchKernel(letkf_piston_kernel(fp64, which), dim3(gx, gy), dim3(kThreads), kargs, 0, s);
}
