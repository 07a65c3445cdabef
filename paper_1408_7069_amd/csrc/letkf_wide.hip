// gfx950 local analyses of the wide shapes: up to 128 members and node patches
// up to 121 nodes (domain size plus twice the halo up to 10 subapertures, up
// to 200 local slopes), past the one-lane-per-member, 64-row layout of
// k_analysis.  The operating point of the paper's timings (Sec. 5.3, Tables
// 1-2: m = 101, 4 x 4 domains with a halo of 2, 128 local slopes) is one.
//
// k_analysis_wide: one 512-thread workgroup (8 wavefronts) per (instance,
// domain) work item.  M = 16 NB is m rounded up to whole 16-column blocks; the
// members past m carry zero anomalies and the padded block of A~ is c I, so
// it does not couple to the others.  Per item (Sec. 4.2):
//   1. node patch of the forecast ensemble (fused form: a X_a + V, Sec.
//      3.1.2), thread = member, four row groups;
//   2. member means in FP64, the weights sqrt(g) = f / sqrt(s r) (taper on
//      Sigma_w^{-1/2}, Sec. 4.1) and the scaled innovation of each local slope;
//   3. the scaled Fried slopes of the anomalies, 16 local slopes at a time,
//      into an FP64 K-major operand, and the Gram on the FP64 matrix cores:
//      wave q accumulates the column block q of A~ = (m-1)/rho I + Y^T Y over
//      the slopes; b = Y^T sqrt(g) d along the way;
//   4.-6. the inverse square root by the P-form Newton-Schulz iteration
//      (the same steps as the 64-member kernel): P_0 = A~ / s with
//      s = ||A~||_F, P_{k+1} = a_k P_k T_k^2, T_k = (3 I - a_k P_k) / 2,
//      carrying V = X' Z (owned rows) and h = Z b, Z = prod sqrt(a_k) T_k,
//      in FP64 (FP32 state with NSP_MIXED: on the FP32 matrix cores once
//      the spectrum's lower bound passes 0.05), the last step second-order
//      once the residual allows; P lives in LDS as its upper block triangle (16 x 16
//      tiles), each wave keeps the column block q of P in registers and
//      forms the column block q of P^2 and of P^3 = P P^2 from it (the right
//      operands stay in registers, the left ones are tiles of P read from
//      LDS, mirrored where below the diagonal);
//   7. owned rows: x_a = x_b + V h / s, X_a = x_a 1^T + sqrt(rho c / s) V,
//      written straight into the global analysis ensemble.
// A work item that meets a non-finite observation or does not converge
// keeps its forecast rows and raises its flag, as in k_analysis.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "letkf_device.h"
#include "letkf_types.h"

namespace letkf {
namespace wide {

constexpr int kW = 8;          // wavefronts per work item
constexpr int kWT = 64 * kW;   // threads per work item
constexpr int kTS = 17;        // row stride of a stored 16 x 16 FP64 tile
constexpr int kTile = 16 * kTS;
// patch-node area (ints): nodes, their packed (i, j), the corner words
constexpr int kPnIj = 128, kPnCw = 256;
// FP64 scratch (offsets in doubles)
constexpr int W_RES = 0;     // 8 waves: partial sums of squares
constexpr int W_H = 8;       // 128: h = Z b
constexpr int W_BP = 136;    // 4 row groups x 128: partial b
constexpr int W_XAM = 648;   // 128: analysis mean of the owned rows
constexpr int W_TOTAL = 776;

// Index of the stored tile (I, J), I <= J, of the upper block triangle.
__host__ __device__ constexpr int tix(int I, int J) { return J * (J + 1) / 2 + I; }

// Sum over the four lanes of one column (lanes c16, c16 + 16, c16 + 32, c16 + 48).
__device__ inline double col_sum(double v) {
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// Layouts of a 16 x 16 tile in the registers of a wavefront (c16 = lane % 16,
// g = lane / 16): element r of a lane is row off(r) of column c16, off(r) =
// g + 4 r for the FP64 16x16x4 accumulator, 4 g + r for the FP32 one.  The
// same off(j) is the contraction index a lane supplies at step j of a
// 16-wide block (FP32: the permuted order 4 g + j), so an accumulator tile is
// the right operand of the next product as it stands.
template <bool F32> __device__ __forceinline__ int off(int g, int r) { return F32 ? 4 * g + r : g + 4 * r; }
template <bool F32> using Acc = typename std::conditional<F32, f32x4, f64x4>::type;
template <bool F32> using Elem = typename std::conditional<F32, float, double>::type;

// The column block q of P in the registers (F32: rounded to FP32) from the
// stored upper triangle.
template <int NB, bool F32>
__device__ __forceinline__ void load_cb(const double *Pp, Acc<F32> (&B)[NB], int q, int lane) {
  const int c16 = lane & 15, g = lane >> 4;
#pragma unroll
  for (int K = 0; K < NB; ++K) {
    const bool up = K <= q;
    const double *t = Pp + (up ? tix(K, q) : tix(q, K)) * kTile;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      B[K][r] = (Elem<F32>)(up ? t[off<F32>(g, r) * kTS + c16] : t[c16 * kTS + off<F32>(g, r)]);
  }
}

// Tiles (I, q), I <= q, of a column block into the stored upper triangle.
template <int NB, bool F32>
__device__ __forceinline__ void store_cb(double *Pp, const Acc<F32> (&C)[NB], int q, int lane) {
  const int c16 = lane & 15, g = lane >> 4;
#pragma unroll
  for (int I = 0; I < NB; ++I)
    if (I <= q) {
      double *t = Pp + tix(I, q) * kTile;
#pragma unroll
      for (int r = 0; r < 4; ++r) t[off<F32>(g, r) * kTS + c16] = (double)C[I][r];
    }
}

// acc[I] += (P R)[16 I.., 16 q..] for every row block I: P the symmetric
// matrix stored as its upper block triangle (left operand, tile (I, K) read
// from the stored (I, K) or, below the diagonal, transposed from (K, I)), R a
// column block in registers (right operand; step j of block K pairs with
// k = 16 K + off(j)).  One pass over K with NB independent accumulators, the
// loads of one step in flight at a time (register pressure); FP32 products
// (operands rounded) with F32.
template <int NB, bool F32>
__device__ __forceinline__ void mm_cb(const double *Pp, const Acc<F32> (&R)[NB], Acc<F32> (&acc)[NB], int lane) {
  const int c16 = lane & 15, g = lane >> 4;
  const int offN = c16 * kTS + off<F32>(g, 0), offT = off<F32>(g, 0) * kTS + c16;
  constexpr int dj = F32 ? 1 : 4;  // step of the contraction index with j
#pragma unroll
  for (int K = 0; K < NB; ++K)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const Elem<F32> b = R[K][j];
#pragma unroll
      for (int I = 0; I < NB; ++I) {
        const double a = I <= K ? Pp[tix(I, K) * kTile + offN + dj * j] : Pp[tix(K, I) * kTile + offT + dj * j * kTS];
        acc[I] = Mfma<Elem<F32>>::mac((Elem<F32>)a, b, acc[I]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
}

// Patch rows [0, r_hi) of X_b for member j (row group rg: rows rg, rg + 4, ..);
// members past m are stored as zero up to M.
template <typename T, bool FUSED>
__device__ __forceinline__ void stage_rows(const AnaArgs<T> &A, const InstDesc &in, const int *pn, uint32_t frame,
                                           T *xs, int XS, int M, int r_hi, int j, int rg) {
  if (j >= M) return;
  const int m = in.m;
  const bool valid = j < m;
  const bool bank = FUSED && A.noise_bank;
  BankDraw bd{};
  if (bank && valid) bd = bank_draw(in, frame, j);
  const T a = (T)in.a, vs = (T)in.vscale;
  for (int r = rg; r < r_hi; r += 4) {
    T v = (T)0;
    if (valid) {
      const int64_t e = in.x_off + (int64_t)pn[r] * m + j;
      const T x = A.x_in[e];
      if constexpr (FUSED) {
        T noise;
        if (bank) {
          const int ij = pn[kPnIj + r];
          noise = (T)bank_value(A.bank, bd, ij & 0xFFFF, ij >> 16);
        } else {
          noise = A.v_in[e];
        }
        v = fma_t(a, x, vs * noise);
      } else {
        v = x;
      }
    }
    xs[r * XS + j] = v;
  }
}

template <typename T, bool FUSED, int NB>
__global__ __launch_bounds__(kWT) void k_analysis_wide(const AnaArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int M = 16 * NB, XS = M + 1, YS = M + 1;
  const int tid = threadIdx.x, q = tid >> 6, lane = tid & 63;
  const int c16 = lane & 15, g = lane >> 4;
  int item = A.order ? A.order[blockIdx.x]
                     : (A.xcd_order ? xcd_item((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x);
  item += A.item_base;
  if (item < 0 || item >= A.n_items) return;
  const DomItem it = A.items[item];
  const InstDesc in = A.inst[it.inst];
  const int m = in.m, np = it.n_patch, nown = it.n_own, nobs = it.n_obs, p = 2 * nobs;
  T *xs = (T *)(smem + A.off_xs);         // patch rows; then V (even steps)
  T *xs1 = (T *)(smem + A.off_clb);       // V (odd steps)
  double *xm = (double *)(smem + A.off_xm);
  double *sg = (double *)(smem + A.off_sg);
  double *dd = (double *)(smem + A.off_dd);
  double *ybm = (double *)(smem + A.off_yb);
  int *pn = (int *)(smem + A.off_pn);
  double *sm = (double *)(smem + A.off_s);
  double *ys = (double *)(smem + A.off_ys);
  double *Pp = (double *)(smem + A.off_u);
  const uint32_t frame = (FUSED && A.noise_bank) ? *A.frame : 0u;
  const double c = (double)(m - 1) / in.rho;
  const int j = tid & 127, rg = tid >> 7;
  const bool act = q < NB;  // the waves that own a column block

  // ---- 1. node patch of X_b ----
  for (int r = tid; r < np; r += kWT) {
    const int gn = A.patch_node[it.patch_off + r];
    pn[r] = gn;
    pn[kPnIj + r] = A.node_ij[2 * (in.node_off + gn)] | (A.node_ij[2 * (in.node_off + gn) + 1] << 16);
  }
  __syncthreads();
  stage_rows<T, FUSED>(A, in, pn, frame, xs, XS, M, np, j, rg);
  __syncthreads();
  for (int r = q; r < np; r += kW) {
    double s = 0.0;
    for (int k = lane; k < m; k += 64) s += (double)xs[r * XS + k];
    s = wave_sum(s);
    if (lane == 0) xm[r] = s / (double)m;
  }
  __syncthreads();

  // ---- 2. weights, slope means and scaled innovation per local slope ----
  int bad = 0;
  for (int o = tid; o < nobs; o += kWT) {
    const uint32_t cw = A.obs_corner[it.obs_off + o];
    pn[kPnCw + o] = (int)cw;
    const int k = A.obs_sub[it.obs_off + o];
    const int ca = cw & 255, cb = (cw >> 8) & 255, cc = (cw >> 16) & 255, cd = cw >> 24;
    const double ybx = 0.5 * ((xm[cb] - xm[ca]) + (xm[cd] - xm[cc]));
    const double yby = 0.5 * ((xm[cc] - xm[ca]) + (xm[cd] - xm[cb]));
    const double f = in.taper_c > 0.0 ? gaspari_cohn(A.obs_dist[it.obs_off + o] / in.taper_c) : 1.0;
    const double rx = A.r_diag[in.y_off + k], ry = A.r_diag[in.y_off + in.n_subaps + k];
    const double sgx = f / sqrt(in.r_scale * rx), sgy = f / sqrt(in.r_scale * ry);
    const double yx = (double)A.y[in.y_off + k], yy = (double)A.y[in.y_off + in.n_subaps + k];
    bad |= !(isfinite(yx) && isfinite(yy));
    sg[o] = sgx;
    sg[nobs + o] = sgy;
    dd[o] = sgx * (yx - ybx);
    dd[nobs + o] = sgy * (yy - yby);
    ybm[o] = ybx;
    ybm[nobs + o] = yby;
  }
  bad = __syncthreads_or(bad);

  // ---- 3. Gram of the scaled slope anomalies and b, 16 slopes a pass ----
  f64x4 acc[NB];
#pragma unroll
  for (int I = 0; I < NB; ++I) acc[I] = Mfma<double>::zero();
  double bp = 0.0;
  for (int c0 = 0; c0 < p; c0 += 16) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int sl = rg + 4 * u, s = c0 + sl;
      double v = 0.0;
      if (s < p && j < m) {
        const bool sx = s < nobs;
        const uint32_t cw = (uint32_t)pn[kPnCw + (sx ? s : s - nobs)];
        const int ca = cw & 255, cb = (cw >> 8) & 255, cc = (cw >> 16) & 255, cd = cw >> 24;
        const double pa = (double)xs[ca * XS + j], pb = (double)xs[cb * XS + j];
        const double pc = (double)xs[cc * XS + j], pd = (double)xs[cd * XS + j];
        const double slope = sx ? 0.5 * ((pb - pa) + (pd - pc)) : 0.5 * ((pc - pa) + (pd - pb));
        v = sg[s] * (slope - ybm[s]);
        bp = fma(v, dd[s], bp);
      }
      if (j < M) ys[sl * YS + j] = v;
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const double bv = ys[(4 * kk + g) * YS + 16 * q + c16];
#pragma unroll
        for (int I = 0; I < NB; ++I) acc[I] = Mfma<double>::mac(ys[(4 * kk + g) * YS + 16 * I + c16], bv, acc[I]);
      }
    }
    __syncthreads();
  }
  sm[W_BP + rg * 128 + j] = bp;
  double ss = 0.0;
  if (act) {
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (16 * I + g + 4 * r == 16 * q + c16) acc[I][r] += c;
        ss = fma(acc[I][r], acc[I][r], ss);
      }
  }
  ss = wave_sum(ss);
  if (lane == 0) sm[W_RES + q] = ss;
  __syncthreads();
  if (tid < M) sm[W_H + tid] = (sm[W_BP + tid] + sm[W_BP + 128 + tid]) + (sm[W_BP + 256 + tid] + sm[W_BP + 384 + tid]);
  double s2 = 0.0;
#pragma unroll
  for (int w = 0; w < kW; ++w) s2 += sm[W_RES + w];
  const double s = sqrt(s2);
  // V_0 = X' of the owned rows in place (rows past n_own, members past m zero);
  // P_0 = A~ / s into the stored upper triangle (over the dead patch rows)
  const int ncbo = (nown + 15) >> 4;
  for (int e = tid; e < 16 * ncbo * M; e += kWT) {
    const int i = e / M, k = e - i * M;
    xs[i * XS + k] = (i < nown && k < m) ? (T)((double)xs[i * XS + k] - xm[i]) : (T)0;
  }
  if (act) {
    const double is = 1.0 / s;
#pragma unroll
    for (int I = 0; I < NB; ++I) acc[I] *= is;
    store_cb<NB, false>(Pp, acc, q, lane);
  }
  __syncthreads();

  // ---- 4.-6. P-form iteration ----
  double *hb = sm + W_H;
  const double tol = A.jtol * 0.01;
  // threshold of the second-order finish (the 64-member kernel's rule)
  const double tol2 = sizeof(T) == 4 ? sqrt(tol) : cbrt(tol * tol);
  const int max_it = A.max_sweeps;
  double l = c / s;
  int nit = 0;
  bool conv = false, finite = isfinite(s);
  // FP32 state with NSP_MIXED: the P updates on the FP32 matrix cores once
  // the spectrum's lower bound passes 0.05 (where the 64-member kernel's
  // first FP32 step starts: its switch rounds P_{k+1} once l_k >= 0.01);
  // P stays in the FP64 triangle (holding FP32 values), the operands rounded
  constexpr bool kF32State = sizeof(T) == 4;
  const double l_switch = A.p32 != 0 ? 0.05 : INFINITY;
  auto step = [&](auto f32tag) {
    constexpr bool F32 = decltype(f32tag)::value;
    using E = Elem<F32>;
    using AC = Acc<F32>;
    using MF = Mfma<E>;
    constexpr int dj = F32 ? 1 : 4;
    const double al = 3.0 / (1.0 + sqrt(l) + l), sa = sqrt(al), ta = 0.5 * al;
    // the diagonal element a lane holds in its column block (tile q, element
    // r with off(r) = c16), made opaque a step so that the selects are formed
    // where used, not kept across the loop in registers
    const int rd = F32 ? c16 - 4 * g : ((c16 - g) >= 0 && ((c16 - g) & 3) == 0 ? (c16 - g) >> 2 : -1);
    int dq = (rd >= 0 && rd < 4) ? 4 * q + rd : -1;
    asm volatile("" : "+v"(dq));
    T *Vc = (nit & 1) ? xs1 : xs, *Vn = (nit & 1) ? xs : xs1;
    AC Pc[NB];
    double e2 = 0.0, th = 0.0, hold = 0.0, q2 = 0.0;
    if (act) {
      load_cb<NB, F32>(Pp, Pc, q, lane);
#pragma unroll
      for (int K = 0; K < NB; ++K)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double d = fma(al, (double)Pc[K][r], 4 * K + r == dq ? -1.0 : 0.0);
          e2 = fma(d, d, e2);
        }
      // V_{k+1} = sqrt(a) V_k T_k on this wave's columns, row block by row block
      for (int cb = 0; cb < ncbo; ++cb) {
        const T *vr = Vc + (16 * cb + c16) * XS + off<F32>(g, 0);
        AC o{};
#pragma unroll
        for (int K = 0; K < NB; ++K)
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            const E tb = (E)fma(-ta, (double)Pc[K][jj], 4 * K + jj == dq ? 1.5 : 0.0);
            o = MF::mac((E)vr[16 * K + dj * jj], tb, o);
          }
#pragma unroll
        for (int r = 0; r < 4; ++r) Vn[(16 * cb + off<F32>(g, r)) * XS + 16 * q + c16] = (T)(sa * (double)o[r]);
      }
      // h_{k+1} = sqrt(a) (3/2 h - ta P h) for row 16 q + c16
      double part = 0.0;
#pragma unroll
      for (int K = 0; K < NB; ++K)
#pragma unroll
        for (int r = 0; r < 4; ++r) part = fma((double)Pc[K][r], hb[16 * K + off<F32>(g, r)], part);
      part = col_sum(part);
      hold = hb[16 * q + c16];
      th = fma(-ta, part, 1.5 * hold);
    }
    e2 = wave_sum(e2);
    if (lane == 0) sm[W_RES + q] = e2;
    const bool more = nit + 1 < max_it;
    AC Qc[NB];
#pragma unroll
    for (int I = 0; I < NB; ++I) Qc[I] = AC{};
    if (act && more) {
      mm_cb<NB, F32>(Pp, Pc, Qc, lane);
      // (P^2 h) for row 16 q + c16, for a second-order finish
#pragma unroll
      for (int K = 0; K < NB; ++K)
#pragma unroll
        for (int r = 0; r < 4; ++r) q2 = fma((double)Qc[K][r], hb[16 * K + off<F32>(g, r)], q2);
      q2 = col_sum(q2);
    }
    __syncthreads();  // #1: residual, P^2 complete; every read of h done
    double d2 = 0.0;
#pragma unroll
    for (int w = 0; w < kW; ++w) d2 += sm[W_RES + w];
    finite = isfinite(d2);
    conv = finite && 0.75 * d2 <= tol;
    // second-order finish (as in the 64-member kernel): sqrt(a) (5/2 X T -
    // 15/8 X + 3/8 a^2 X P^2) for X = V, h, once the residual is below tol2
    const bool fin2 = finite && !conv && more && 0.75 * d2 <= tol2;
    ++nit;
    if (fin2) {
      const double c2 = 0.375 * al * al;
      if (act) {
        for (int cb = 0; cb < ncbo; ++cb) {
          const T *vr = Vc + (16 * cb + c16) * XS + off<F32>(g, 0);
          AC o{};
#pragma unroll
          for (int K = 0; K < NB; ++K)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) o = MF::mac((E)vr[16 * K + dj * jj], Qc[K][jj], o);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int e = (16 * cb + off<F32>(g, r)) * XS + 16 * q + c16;
            // Vn holds sqrt(a) V T (this wave's columns, written by it)
            Vn[e] = (T)fma(sa * c2, (double)o[r], fma(2.5, (double)Vn[e], -1.875 * sa * (double)Vc[e]));
          }
        }
        if (g == 0) hb[16 * q + c16] = sa * fma(c2, q2, fma(2.5, th, -1.875 * hold));
      }
      conv = true;
    } else if (act && g == 0) {
      hb[16 * q + c16] = sa * th;
    }
    if (!conv && finite && more) {
      // P_{k+1} = a (9/4 P - 3/2 a P^2 + 1/4 a^2 P^3), P^3 = P P^2 (P read
      // from LDS, P^2's column block from the registers), accumulated over
      // P's own column block: two blocks live at a time
      if (act) {
        const E i2 = (E)(1.0 / (al * al)), a6 = (E)(6.0 * al), f3 = (E)(0.25 * al * al * al);
#pragma unroll
        for (int K = 0; K < NB; ++K) Pc[K] = ((E)9 * Pc[K] - a6 * Qc[K]) * i2;
        mm_cb<NB, F32>(Pp, Qc, Pc, lane);
#pragma unroll
        for (int K = 0; K < NB; ++K) Pc[K] *= f3;
      }
      __syncthreads();  // #2: every read of P_k done
      if (act) store_cb<NB, F32>(Pp, Pc, q, lane);
    }
    __syncthreads();  // P_{k+1}, V and h complete
    l = al * l * (3.0 - al * l) * (3.0 - al * l) * 0.25;
  };
  while (finite) {
    if (kF32State && l >= l_switch)
      step(std::true_type{});
    else
      step(std::false_type{});
    if (conv || nit >= max_it) break;
  }
  const bool keep = bad || !finite || !conv;
  if (tid == 0) A.flags[item] = (bad || !finite ? 1 : 0) | (conv || !finite ? 0 : 2) | (min(nit, 255) << 8);
  if (keep) {
    // the forecast is the result: the owned rows of X_b again
    stage_rows<T, FUSED>(A, in, pn, frame, xs, XS, M, nown, j, rg);
    __syncthreads();
    for (int i = q; i < nown; i += kW)
      for (int k = lane; k < m; k += 64) A.x_out[in.x_off + (int64_t)pn[i] * m + k] = xs[i * XS + k];
    if (tid < nown && A.x_mean) A.x_mean[in.node_off + pn[tid]] = (T)xm[tid];
    return;
  }
  // ---- 7. x_a = x_b + V h / s, X_a = x_a 1^T + sqrt(rho c / s) V ----
  const T *V = (nit & 1) ? xs1 : xs;
  for (int i = q; i < nown; i += kW) {
    double v = 0.0;
    for (int k = lane; k < m; k += 64) v = fma((double)V[i * XS + k], hb[k], v);
    v = wave_sum(v);
    if (lane == 0) sm[W_XAM + i] = xm[i] + v / s;
  }
  __syncthreads();
  const double wsc = sqrt(in.rho * c / s);
  for (int i = q; i < nown; i += kW)
    for (int k = lane; k < m; k += 64)
      A.x_out[in.x_off + (int64_t)pn[i] * m + k] = (T)(sm[W_XAM + i] + wsc * (double)V[i * XS + k]);
  if (tid < nown && A.x_mean) A.x_mean[in.node_off + pn[tid]] = (T)sm[W_XAM + tid];
}

template <typename T, int NB> static const void *kernel_nb(int fused) {
  return fused ? (const void *)k_analysis_wide<T, true, NB> : (const void *)k_analysis_wide<T, false, NB>;
}

template <typename T> static const void *kernel_of(int fused, int nb) {
  switch (nb) {
    case 4: return kernel_nb<T, 4>(fused);
    case 5: return kernel_nb<T, 5>(fused);
    case 6: return kernel_nb<T, 6>(fused);
    case 7: return kernel_nb<T, 7>(fused);
    case 8: return kernel_nb<T, 8>(fused);
    default: return nullptr;
  }
}

}  // namespace wide
}  // namespace letkf

// The wide-shape analysis kernel of NB 16-column blocks (4 <= NB <= 8), NULL otherwise.
extern "C" const void *letkf_wide_kernel(int fp64, int fused, int nb) {
  using namespace letkf::wide;
  return fp64 ? kernel_of<double>(fused, nb) : kernel_of<float>(fused, nb);
}

extern "C" int letkf_wide_threads(void) { return letkf::wide::kWT; }

// LDS scratch of the wide kernel (doubles), its patch-node area (ints) and the
// bytes of its stored upper block triangle of NB blocks.
extern "C" size_t letkf_wide_scratch_doubles(void) { return letkf::wide::W_TOTAL; }
extern "C" size_t letkf_wide_pn_ints(void) { return 384; }
extern "C" size_t letkf_wide_tri_bytes(int nb) {
  return (size_t)(nb * (nb + 1) / 2) * letkf::wide::kTile * sizeof(double);
}
