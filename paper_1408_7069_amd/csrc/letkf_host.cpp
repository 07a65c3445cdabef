// Host side of libletkf: geometry planner, device state, launches, C ABI.
//
// Geometry (planned once per instance at letkf_create):
//  * valid subapertures: > 50 % of the area inside the annulus eps N/2 <= r <= N/2
//    (Sec. 5), sampled 64 x 64 with exact integer radii, or a caller mask;
//  * valid nodes: corners of valid subapertures (Fried geometry, App. B),
//    numbered row-major; slopes [x of valid subapertures; y same order];
//  * domains: b x b subaperture blocks owning the nodes (i, j) with
//    (min(i / b, nb - 1), min(j / b, nb - 1)), nb = ceil(N / b); observation
//    region = the block grown by h subapertures (Sec. 4.1);
//  * per domain, a node patch (owned nodes first, then the other corners of
//    the region's subapertures) that the analysis kernel loads into LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/letkf.h"
#include "letkf_types.h"

using namespace letkf;

extern "C" hipError_t letkf_launch_analysis(const void *args, int fp64, int fused, int eig, int grid,
                                            size_t lds, hipStream_t s);
extern "C" const void *letkf_analysis_kernel(int fp64, int fused, int eig);
extern "C" const void *letkf_command_kernel(int fp64);
extern "C" hipError_t letkf_launch_command(int fp64, const InstDesc *insts, int n_inst, int max_nodes,
                                           const void *x, void *u1, void *u2, hipStream_t s);
extern "C" const void *letkf_copy_kernel(int fp64);
extern "C" const void *letkf_refit_sums_kernel(int fp64);
extern "C" const void *letkf_blend_rhs_kernel(void);
extern "C" const void *letkf_blend_solve_kernel(void);
extern "C" const void *letkf_blend_gather_kernel(int fp64);
extern "C" hipError_t letkf_launch_blend(int fp64, const InstDesc *insts, const DomItem *items, int n_items,
                                         const int32_t *patch_node, const double *smean, const int32_t *boff,
                                         const int32_t *bent, const int32_t *bitem, const double *bw,
                                         const int32_t *dom_base, const int64_t *minv_off, const double *minv,
                                         double *rhs, double *pi, const void *stage, void *x, uint32_t *frame,
                                         int max_nodes, int n_inst, hipStream_t s);
extern "C" const void *letkf_refit_finish_kernel(void);
extern "C" int letkf_refit_stride(int max_nodes);
extern "C" hipError_t letkf_launch_refit(int fp64, void *insts, void *rs, const void *x_now, const void *x_prev,
                                         double *part, int max_nodes, int n_inst, hipStream_t s);
extern "C" hipError_t letkf_launch_copy(int fp64, const void *src, void *dst, int64_t n, hipStream_t s);
extern "C" hipError_t letkf_launch_forecast(int fp64, const InstDesc *insts, int n_inst,
                                            const int32_t *node_ij, const void *xa, const void *v,
                                            const float *bank, const uint32_t *frame, void *xb,
                                            const void *xprev,
                                            int64_t max_elems, hipStream_t s);
extern "C" hipError_t letkf_launch_frame_advance(uint32_t *frame, hipStream_t s);
extern "C" const void *letkf_frame_advance_kernel(void);
extern "C" hipError_t letkf_launch_slopes(int fp64, const InstDesc *insts, int n_inst,
                                          const int32_t *subap_nodes, const void *phase,
                                          void *slopes, int max_subaps, hipStream_t s);
extern "C" hipError_t letkf_launch_mean(int fp64, const InstDesc *insts, int n_inst, const void *x,
                                        void *mean, int max_nodes, hipStream_t s);
extern "C" hipError_t letkf_launch_eigh(const double *A, int m, int batch, double tol,
                                        int max_sweeps, double *Q, double *lam, int32_t *sweeps,
                                        hipStream_t s);
extern "C" size_t letkf_args_size(int fp64);
extern "C" int letkf_analysis_threads(void);
extern "C" int letkf_analysis_threads_for(int eig);
extern "C" size_t letkf_wide_scratch_doubles(void);
extern "C" size_t letkf_wide_pn_ints(void);
extern "C" size_t letkf_wide_tri_bytes(int nb);
extern "C" size_t letkf_resvar_stats_doubles(int n_inst);
extern "C" size_t letkf_analysis_scratch_doubles(void);
extern "C" size_t letkf_analysis_fwd_scratch_doubles(void);
extern "C" size_t letkf_analysis_xch_bytes(void);
extern "C" const void *letkf_adjoint_kernel(int fp64);
extern "C" size_t letkf_adjoint_scratch_doubles(void);
extern "C" size_t letkf_adjoint_args_size(int fp64);
extern "C" hipError_t letkf_launch_adjoint(int fp64, const void *args, int grid, size_t lds,
                                           hipStream_t s);
extern "C" hipError_t letkf_launch_adjoint_nodes(int fp64, const InstDesc *insts, int n_inst,
                                                 const int32_t *node_adj, const int32_t *slot_off,
                                                 const int32_t *slots, const void *xpbar,
                                                 const double *xbbar, const void *ybar,
                                                 const double *dbar, void *xbar_out, int max_nodes,
                                                 hipStream_t s);
extern "C" hipError_t letkf_launch_resvar(int fp64, const InstDesc *insts, int n_inst, const void *x,
                                          const void *truth, const double *weights, double *stats,
                                          double *acc, hipStream_t s);
extern "C" hipError_t letkf_launch_resvar_adjoint(int fp64, const InstDesc *insts, int n_inst,
                                                  const void *x, const void *truth,
                                                  const double *weights, const double *stats,
                                                  void *xbar, int max_nodes, hipStream_t s);
extern "C" const void *letkf_piston_kernel(int fp64, int which);
extern "C" size_t letkf_piston_args_size(int fp64);
extern "C" const void *letkf_piston_finish_kernel(int fp64);
extern "C" hipError_t letkf_launch_piston_finish(int fp64, const void *args, int n_items,
                                                 uint32_t *frame, hipStream_t s);
extern "C" void letkf_piston_grid(int which, int n_items, int n_inst, int max_nodes, int64_t max_elems,
                                  int *gx, int *gy);
extern "C" hipError_t letkf_launch_piston(int fp64, int which, const void *args, int gx, int gy,
                                          hipStream_t s);
extern "C" size_t letkf_noalloc_scratch_bytes(void);
extern "C" hipError_t letkf_noalloc_scratch(int device, void **ptr);
extern "C" hipError_t letkf_launch_theta_sum(const int32_t *dom_base, int n_inst, const double *theta,
                                             double *theta_acc, hipStream_t s);

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

#define HIPCHK(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(LETKF_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_));      \
  } while (0)

// Mirror of the kernel argument block (layout must match AnaArgs<T>).
template <typename T> struct AnaArgsHost {
  const InstDesc *inst;
  const DomItem *items;
  int32_t item_base, n_items, xcd_order, noise_bank;
  const int32_t *patch_node;
  const uint32_t *obs_corner;
  const int32_t *obs_sub;
  const double *obs_dist;
  const int32_t *node_ij;
  const double *r_diag;
  const T *x_in;
  const T *v_in;
  const float *bank;
  const T *y;
  T *x_out;
  T *x_mean;
  int32_t *flags;
  const uint32_t *frame;
  const T *u_prev2;
  const T *x_prev;
  T *stage;
  double *stage_mean;
  double jtol;
  int32_t max_sweeps;
  int32_t off_xs, off_xm, off_sg, off_dd, off_yb, off_pn, off_s, off_u, off_ys;
  int32_t off_clb, off_clr;
  int32_t round_items;
  int32_t p32;
  const int32_t *order;  // grid slot -> work item (-1: none), or NULL
};

// Mirror of PistonArgs<T>.
template <typename T> struct PistonArgsHost {
  const InstDesc *inst;
  const DomItem *items;
  int32_t n_items, pad0;
  const int32_t *patch_node;
  const int32_t *node_adj;
  const int32_t *subap_nodes;
  const int32_t *owner_item;
  const int32_t *dom_base;
  const int64_t *minv_off;
  const double *minv;
  const T *x_mean;
  const T *y;
  double *rhs;
  double *pi;
  T *x;
  const int32_t *term_off;
  const PistonTerm *terms;
  const PistonItem *pitem;
};

// Mirror of AdjArgs<T>.
template <typename T> struct AdjArgsHost {
  AnaArgsHost<T> F;
  const T *xbar;
  T *xpbar;
  double *xbbar;
  T *ybar;
  double *dbar;
  double *theta;
  uint32_t frame;
  int32_t off_q, off_sa;
};

// Whether the host mirrors of the kernel argument blocks have the kernels'
// sizes: 0, else the first block that differs (1 analysis, 2 adjoint, 3
// piston).  The kernels and this file are separate translation units, so a
// field added on one side only is caught here rather than read shifted.
extern "C" int letkf_layout_check(void) {
  if (sizeof(AnaArgsHost<float>) != letkf_args_size(0) || sizeof(AnaArgsHost<double>) != letkf_args_size(1))
    return 1;
  if (sizeof(AdjArgsHost<float>) != letkf_adjoint_args_size(0) ||
      sizeof(AdjArgsHost<double>) != letkf_adjoint_args_size(1))
    return 2;
  if (sizeof(PistonArgsHost<float>) != letkf_piston_args_size(0) ||
      sizeof(PistonArgsHost<double>) != letkf_piston_args_size(1))
    return 3;
  return 0;
}

struct InstGeom {
  int N = 0, b = 0, h = 0, m = 0;
  std::vector<uint8_t> mask;           // N*N
  std::vector<int32_t> node_index;     // (N+1)^2, -1 invalid
  std::vector<int32_t> node_ij;        // 2 n
  std::vector<int32_t> subaps;         // 2 p_sap (i, j)
  std::vector<int32_t> subap_nodes;    // 4 p_sap
  int n_nodes = 0, n_subaps = 0;
  // domains
  std::vector<std::array<int, 2>> blocks;
  std::vector<std::vector<int32_t>> owned, patch, obs_sub;
  std::vector<std::vector<uint32_t>> obs_corner;
  std::vector<std::vector<double>> obs_dist;
  std::vector<int32_t> owner;          // n
};

}  // namespace

struct letkf_handle {
  int device = 0;
  int fp64 = 0;
  size_t esize = 4;
  int n_inst = 0;
  std::vector<InstGeom> geom;
  std::vector<InstDesc> desc;
  std::vector<DomItem> items;
  std::vector<int32_t> dom_base;  // first global domain number of each instance
  int64_t total_x = 0, total_y = 0, total_nodes = 0, total_obs = 0;
  int max_patch = 0, max_obs_sub = 0, max_own = 0, max_m = 0, max_subaps = 0, max_nodes = 0;
  int64_t max_elems = 0;
  bool any_bank = false, all_bank = true;
  double jtol = 0.0;
  int max_sweeps = 30;
  int transform = LETKF_TRANSFORM_NS64;  // forward transform (FP64 handles: never NS32)
  bool wide = false;  // shapes past the 64-member, 64-node layout: the wide analysis kernel
  bool wide_p32 = false;  // the wide analysis with FP32 state asked for NSP_MIXED
  size_t lds = 0;
  int32_t off[9] = {0};      // LDS layout of the adjoint's forward stages
  int32_t fwd_off[9] = {0};  // LDS layout of the analysis
  int32_t cl_off[2] = {0, 0};  // covariance localisation: offsets of B and of the solve's columns
  int32_t round_items = 32;   // work items of one dispatch round per XCD (the CUs of one XCD)
  // device
  InstDesc *d_desc = nullptr;
  DomItem *d_items = nullptr;
  int32_t *d_patch = nullptr, *d_obs_sub = nullptr, *d_node_ij = nullptr, *d_subap_nodes = nullptr;
  uint32_t *d_obs_corner = nullptr;
  double *d_obs_dist = nullptr;
  float *d_bank = nullptr;
  double *d_r = nullptr;
  void *d_xa[2] = {nullptr, nullptr};
  void *d_xb = nullptr;
  void *d_tmp = nullptr;  // mean scratch
  uint32_t *d_frame = nullptr;
  int32_t *d_flags = nullptr;
  int cur = 0;
  bool have_xb = false;
  // graph replay of the fused frame, one per ping-pong parity
  int use_graph = 1, xcd_order = 1;  // xcd_order: the item order, LETKF_ORDER_*
  int32_t *d_order = nullptr;         // slot -> item table of LETKF_ORDER_XCD_PAIRED
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  hipGraphNode_t gnode[2] = {nullptr, nullptr};
  std::vector<unsigned char> gargs[2];
  // adjoint: node -> subaperture roles, per-subaperture slot lists, item
  // ranges per instance, LDS layout, and buffers allocated on first use
  size_t adj_lds = 0;
  int32_t adj_off[2] = {0, 0};
  bool adj_ok = false;
  int32_t *d_node_adj = nullptr, *d_slot_off = nullptr, *d_slots = nullptr, *d_dom_base = nullptr;
  double *d_ones = nullptr, *d_stats = nullptr;
  void *d_xpbar = nullptr, *d_ybar = nullptr;
  double *d_xbbar = nullptr, *d_dbar = nullptr, *d_theta = nullptr;
  // differential pistons: per-instance M^+ and the work buffers
  bool any_piston = false;
  bool any_loop = false;           // an instance runs the closed-loop model
  bool any_ar2 = false;            // an instance has an AR(2) model
  bool any_refit = false;          // an instance refits its AR(1) model online
  void *d_xprev = nullptr;         // AR(2) / refit: the analysis ensemble of the frame before the current one
  RefitState *d_refit = nullptr;   // refit sums and settings per instance
  bool any_blend = false;          // an instance gathers in blend mode
  void *d_stage = nullptr;         // blend: analysed patch rows [patch entry][64]
  double *d_smean = nullptr;       // blend: their member means
  int32_t *d_boff = nullptr, *d_bent = nullptr, *d_bitem = nullptr;  // blend: node -> patch entries
  double *d_bw = nullptr;          // blend: normalised weights of those entries
  double *d_rpart = nullptr;       // refit partial sums [instance][stride][4]
  void *d_u1 = nullptr, *d_u2 = nullptr;  // commands u_{k-1}, u_{k-2} per node
  int32_t *d_owner_item = nullptr;
  int64_t *d_minv_off = nullptr;
  double *d_minv = nullptr, *d_prhs = nullptr, *d_pi = nullptr;
  int32_t *d_pterm_off = nullptr;  // piston right-hand-side terms per item
  PistonTerm *d_pterms = nullptr;
  PistonItem *d_pitem = nullptr;   // per item: what the piston step reads
  bool pterm_fixed = false;        // terms at a fixed stride of 64 an item
  void *d_xmean = nullptr;
  std::vector<unsigned char> gpargs[2][2];  // graph: rhs args, solve/apply args
  hipGraphNode_t gpnode[2][3] = {};
  // optional HIP-event timing of the analysis launches of direct steps
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> tev;
  size_t tev_used = 0;
};

namespace {

// ---------------------------------------------------------------- geometry
std::vector<uint8_t> annulus_mask(int N, double eps) {
  const int ss = 64;
  const int64_t outer = (int64_t)ss * N * (int64_t)ss * N;
  const double inner = (eps * N * ss) * (eps * N * ss);
  std::vector<uint8_t> mask((size_t)N * N, 0);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      int lit = 0;
      for (int t = 0; t < ss; ++t) {
        const int64_t Y = 2LL * ss * i + 2 * t + 1 - (int64_t)ss * N;
        for (int u = 0; u < ss; ++u) {
          const int64_t X = 2LL * ss * j + 2 * u + 1 - (int64_t)ss * N;
          const int64_t r2 = X * X + Y * Y;
          if (r2 <= outer && (double)r2 >= inner) ++lit;
        }
      }
      mask[(size_t)i * N + j] = 2 * lit > ss * ss;
    }
  return mask;
}

int plan_instance(const letkf_config &c, InstGeom &g, std::string &err) {
  const int N = c.n_sub;
  g.N = N;
  g.b = c.domain_size;
  g.h = c.halo;
  g.m = c.m;
  g.mask = c.subap_mask ? std::vector<uint8_t>(c.subap_mask, c.subap_mask + (size_t)N * N)
                        : annulus_mask(N, c.obscuration);
  for (auto &v : g.mask) v = v ? 1 : 0;
  const int N1 = N + 1;
  std::vector<uint8_t> nv((size_t)N1 * N1, 0);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j)
      if (g.mask[(size_t)i * N + j])
        nv[i * N1 + j] = nv[(i + 1) * N1 + j] = nv[i * N1 + j + 1] = nv[(i + 1) * N1 + j + 1] = 1;
  g.node_index.assign((size_t)N1 * N1, -1);
  int k = 0;
  for (int i = 0; i < N1; ++i)
    for (int j = 0; j < N1; ++j)
      if (nv[i * N1 + j]) {
        g.node_index[i * N1 + j] = k++;
        g.node_ij.push_back(i);
        g.node_ij.push_back(j);
      }
  g.n_nodes = k;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j)
      if (g.mask[(size_t)i * N + j]) {
        g.subaps.push_back(i);
        g.subaps.push_back(j);
        g.subap_nodes.push_back(g.node_index[i * N1 + j]);
        g.subap_nodes.push_back(g.node_index[i * N1 + j + 1]);
        g.subap_nodes.push_back(g.node_index[(i + 1) * N1 + j]);
        g.subap_nodes.push_back(g.node_index[(i + 1) * N1 + j + 1]);
      }
  g.n_subaps = (int)(g.subaps.size() / 2);
  if (g.n_subaps == 0) {
    err = "instance has no valid subaperture";
    return LETKF_E_INVAL;
  }
  std::vector<int32_t> sub_id((size_t)N * N, -1);
  for (int q = 0; q < g.n_subaps; ++q) sub_id[g.subaps[2 * q] * N + g.subaps[2 * q + 1]] = q;
  // domains
  const int b = g.b, h = g.h, nb = (N + b - 1) / b;
  std::vector<std::vector<int32_t>> blk_nodes((size_t)nb * nb);
  g.owner.assign(g.n_nodes, -1);
  for (int n = 0; n < g.n_nodes; ++n) {
    const int i = g.node_ij[2 * n], j = g.node_ij[2 * n + 1];
    const int I = std::min(i / b, nb - 1), J = std::min(j / b, nb - 1);
    blk_nodes[I * nb + J].push_back(n);
  }
  for (int I = 0; I < nb; ++I)
    for (int J = 0; J < nb; ++J) {
      auto &own = blk_nodes[I * nb + J];
      if (own.empty()) continue;
      const int d = (int)g.owned.size();
      for (int n : own) g.owner[n] = d;
      g.blocks.push_back({I, J});
      g.owned.push_back(own);  // ascending: nodes were visited in index order
      std::vector<int32_t> obs;
      const int i0 = std::max(I * b - h, 0), i1 = std::min(std::min((I + 1) * b, N) + h, N);
      const int j0 = std::max(J * b - h, 0), j1 = std::min(std::min((J + 1) * b, N) + h, N);
      for (int i = i0; i < i1; ++i)
        for (int j = j0; j < j1; ++j)
          if (sub_id[i * N + j] >= 0) obs.push_back(sub_id[i * N + j]);
      // patch: owned first, then the other corners (ascending)
      std::vector<int32_t> patch = own;
      std::vector<int32_t> extra;
      for (int q : obs)
        for (int t = 0; t < 4; ++t) {
          const int nd = g.subap_nodes[4 * q + t];
          if (g.owner[nd] != d || std::find(own.begin(), own.end(), nd) == own.end())
            extra.push_back(nd);
        }
      std::sort(extra.begin(), extra.end());
      extra.erase(std::unique(extra.begin(), extra.end()), extra.end());
      for (int nd : extra)
        if (std::find(own.begin(), own.end(), nd) == own.end()) patch.push_back(nd);
      if (patch.size() > (size_t)kMaxPatchWide || obs.size() > (size_t)kMaxObsSubWide) {
        err = "domain patch exceeds 128 nodes or 100 observation subapertures";
        return LETKF_E_INVAL;
      }
      std::vector<uint32_t> corners;
      std::vector<double> dist;
      for (int q : obs) {
        uint32_t w = 0;
        for (int t = 0; t < 4; ++t) {
          const int nd = g.subap_nodes[4 * q + t];
          const int loc = (int)(std::find(patch.begin(), patch.end(), nd) - patch.begin());
          w |= (uint32_t)loc << (8 * t);
        }
        corners.push_back(w);
        const double dy = g.subaps[2 * q] + 0.5 - (I + 0.5) * b;
        const double dx = g.subaps[2 * q + 1] + 0.5 - (J + 0.5) * b;
        dist.push_back(std::sqrt(dy * dy + dx * dx));
      }
      g.patch.push_back(patch);
      g.obs_sub.push_back(obs);
      g.obs_corner.push_back(corners);
      g.obs_dist.push_back(dist);
    }
  return LETKF_OK;
}

int pinv_by_components(std::vector<double> &M, int nd, std::vector<double> &out, std::string &err,
                       const char *what);

// Tent weight of patch node n in domain d for the blend-mode gather:
// t(d_i) t(d_j), t(d) = 1 - d / (h + 2), d_i (d_j) the distance in node pitches
// of the node's row (column) from the rows (columns) of the domain's block (the
// last block row and column run to the grid edge).
double blend_weight(const InstGeom &g, int d, int n) {
  const int nb = (g.N + g.b - 1) / g.b;
  double w = 1.0;
  for (int ax = 0; ax < 2; ++ax) {
    const int K = g.blocks[d][ax], v = g.node_ij[2 * n + ax];
    const int lo = K * g.b, hi = K == nb - 1 ? g.N : (K + 1) * g.b - 1;
    const int dist = std::max(0, std::max(lo - v, v - hi));
    w *= 1.0 - dist / (g.h + 2.0);
  }
  return w;
}

// L^+ of the blend alignment of one instance: L is the graph Laplacian of the
// domains weighted by the number of nodes their patches share (for every node
// and every ordered pair of distinct patches holding it: L_ll += 1,
// L_lq -= 1).
int blend_minv(const InstGeom &g, std::vector<double> &out, std::string &err) {
  const int nd = (int)g.owned.size();
  if (nd > 4096) {
    err = "the blend-mode gather supports at most 4096 domains per instance";
    return LETKF_E_INVAL;
  }
  std::vector<std::vector<int>> holders((size_t)g.n_nodes);
  for (int d = 0; d < nd; ++d)
    for (int32_t n : g.patch[d]) holders[n].push_back(d);
  std::vector<double> M((size_t)nd * nd, 0.0);
  for (const auto &hs : holders)
    for (int l : hs)
      for (int q : hs)
        if (q != l) {
          M[(size_t)l * nd + l] += 1.0;
          M[(size_t)l * nd + q] -= 1.0;
        }
  return pinv_by_components(M, nd, out, err, "blend alignment");
}

// M^+ of the differential-piston fit of one instance, row-major nd x nd:
// M = P^T D^T D P (P: node -> owning domain); the common piston of a
// connected set of domains is not measurable and the right-hand sides are
// orthogonal to it (pinv_by_components).
int piston_minv(const InstGeom &g, std::vector<double> &out, std::string &err) {
  const int nd = (int)g.owned.size();
  if (nd > 4096) {
    err = "differential-piston removal supports at most 4096 domains per instance";
    return LETKF_E_INVAL;
  }
  std::vector<double> M((size_t)nd * nd, 0.0);
  const double cx[4] = {-0.5, 0.5, -0.5, 0.5}, cy[4] = {-0.5, -0.5, 0.5, 0.5};
  for (int q = 0; q < g.n_subaps; ++q) {
    const int32_t *cn = &g.subap_nodes[4 * q];
    for (int comp = 0; comp < 2; ++comp) {
      int dl[4];
      double cv[4];
      int n = 0;
      for (int t = 0; t < 4; ++t) {
        const int d = g.owner[cn[t]];
        int k = 0;
        while (k < n && dl[k] != d) ++k;
        if (k == n) {
          dl[n] = d;
          cv[n++] = 0.0;
        }
        cv[k] += comp ? cy[t] : cx[t];
      }
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) M[(size_t)dl[a] * nd + dl[b]] += cv[a] * cv[b];
    }
  }
  return pinv_by_components(M, nd, out, err, "differential-piston");
}

// Pseudo-inverse of a symmetric positive semi-definite nd x nd matrix whose
// null space is the constant vector on each connected set of domains (the
// sets from its nonzero off-diagonal entries): mu is added on every set to
// make it definite, then it is inverted through its Cholesky factor.  Applied
// to right-hand sides with zero sum on every set this gives the minimum-norm
// least-squares solution.  M is overwritten.
int pinv_by_components(std::vector<double> &M, int nd, std::vector<double> &out, std::string &err,
                       const char *what) {
  std::vector<int> comp(nd);
  for (int d = 0; d < nd; ++d) comp[d] = d;
  std::function<int(int)> root = [&](int d) { return comp[d] == d ? d : (comp[d] = root(comp[d])); };
  for (int d = 0; d < nd; ++d)
    for (int e = d + 1; e < nd; ++e)
      if (M[(size_t)d * nd + e] != 0.0) comp[root(d)] = root(e);
  std::map<int, std::vector<int>> sets;
  for (int d = 0; d < nd; ++d) sets[root(d)].push_back(d);
  for (auto &kv : sets) {
    double dmax = 0.0;
    for (int d : kv.second) dmax = std::max(dmax, M[(size_t)d * nd + d]);
    const double mu = dmax > 0.0 ? dmax / (double)kv.second.size() : 1.0;
    for (int d : kv.second)
      for (int e : kv.second) M[(size_t)d * nd + e] += mu;
  }
  // Cholesky M = L L^T (lower, in place)
  for (int j = 0; j < nd; ++j) {
    double djj = M[(size_t)j * nd + j];
    for (int k = 0; k < j; ++k) djj -= M[(size_t)j * nd + k] * M[(size_t)j * nd + k];
    if (!(djj > 0.0)) {
      err = std::string(what) + " normal matrix is not definite";
      return LETKF_E_INVAL;
    }
    const double ljj = std::sqrt(djj);
    M[(size_t)j * nd + j] = ljj;
    for (int i = j + 1; i < nd; ++i) {
      double v = M[(size_t)i * nd + j];
      for (int k = 0; k < j; ++k) v -= M[(size_t)i * nd + k] * M[(size_t)j * nd + k];
      M[(size_t)i * nd + j] = v / ljj;
    }
  }
  // inverse column by column: L z = e_c, L^T x = z
  out.assign((size_t)nd * nd, 0.0);
  std::vector<double> z(nd);
  for (int c = 0; c < nd; ++c) {
    for (int i = 0; i < nd; ++i) {
      double v = i == c ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) v -= M[(size_t)i * nd + k] * z[k];
      z[i] = v / M[(size_t)i * nd + i];
    }
    for (int i = nd - 1; i >= 0; --i) {
      double v = z[i];
      for (int k = i + 1; k < nd; ++k) v -= M[(size_t)k * nd + i] * out[(size_t)k * nd + c];
      out[(size_t)i * nd + c] = v / M[(size_t)i * nd + i];
    }
  }
  return LETKF_OK;
}

int validate(const letkf_config &c, int idx, std::string &err) {
  std::ostringstream o;
  o << "instance " << idx << ": ";
  if (c.n_sub < 1 || c.n_sub > 4096) err = o.str() + "n_sub out of range";
  else if (c.m < 2 || c.m > kMaxMembers) err = o.str() + "m must be in [2, 128]";
  else if (c.domain_size < 1) err = o.str() + "domain_size must be >= 1";
  else if (c.halo < 0) err = o.str() + "halo must be >= 0";
  else if (c.domain_size + 2 * c.halo > 10) err = o.str() + "domain_size + 2*halo must be <= 10";
  else if (!(c.rho > 0)) err = o.str() + "rho must be > 0";
  else if (!(c.r_scale > 0)) err = o.str() + "r_scale must be > 0";
  else if (!c.r_diag && !(c.r_sigma2 > 0)) err = o.str() + "r_sigma2 must be > 0";
  else if (!(c.taper_c >= 0)) err = o.str() + "taper_c must be >= 0";
  else if (!c.subap_mask && !(c.obscuration >= 0 && c.obscuration < 1)) err = o.str() + "obscuration must be in [0, 1)";
  else if (c.precision != LETKF_FP32 && c.precision != LETKF_FP64) err = o.str() + "unknown precision";
  else if (c.model != LETKF_MODEL_PHASE && c.model != LETKF_MODEL_CLOSED_LOOP) err = o.str() + "unknown model";
  else if (!(std::fabs(c.ar2_coeff) < 1.0)) err = o.str() + "ar2_coeff must be in (-1, 1)";
  else if (c.ar2_coeff != 0.0 && c.model != LETKF_MODEL_PHASE)
    err = o.str() + "the AR(2) model runs with the delay-free phase state only";
  else if (!(c.refit_forgetting >= 0.0 && c.refit_forgetting <= 1.0))
    err = o.str() + "refit_forgetting must be in [0, 1]";
  else if (c.refit_forgetting > 0.0 && c.ar2_coeff != 0.0) err = o.str() + "the online refit fits the AR(1) model only";
  else if (c.refit_forgetting > 0.0 && !(c.ar_coeff >= 0.0 && c.ar_coeff < 1.0))
    err = o.str() + "the online refit needs ar_coeff in [0, 1)";
  else if (c.gather_mode != LETKF_GATHER_CONCAT && c.gather_mode != LETKF_GATHER_BLEND)
    err = o.str() + "unknown gather_mode";
  else if (c.localisation != LETKF_LOCALISATION_DOMAIN && c.localisation != LETKF_LOCALISATION_COVARIANCE)
    err = o.str() + "unknown localisation";
  else if (c.localisation == LETKF_LOCALISATION_COVARIANCE && c.gather_mode == LETKF_GATHER_BLEND)
    err = o.str() + "covariance localisation updates the owned rows only: no blend-mode gather";
  else if (c.localisation == LETKF_LOCALISATION_COVARIANCE && c.model != LETKF_MODEL_PHASE)
    err = o.str() + "covariance localisation runs with the delay-free phase state only";
  else if (c.gather_mode == LETKF_GATHER_BLEND && c.piston_removal)
    err = o.str() + "the blend-mode gather aligns the patch pistons itself: piston_removal must be off";
  else if (c.noise_bank && (c.bank_screens < 1 || c.bank_side < c.n_sub + 1 ||
                            (c.bank_side & (c.bank_side - 1)) != 0))
    err = o.str() + "noise bank needs >= 1 screen and a power-of-two side >= N + 1";
  else return LETKF_OK;
  return LETKF_E_INVAL;
}

template <typename T> int to_device(T **dst, const std::vector<T> &src) {
  const size_t bytes = std::max<size_t>(1, src.size()) * sizeof(T);
  hipError_t e = hipMalloc((void **)dst, bytes);
  if (e != hipSuccess) return fail(LETKF_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  if (!src.empty()) HIPCHK(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return LETKF_OK;
}

size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

void free_handle(letkf_handle *h) {
  if (!h) return;
  hipSetDevice(h->device);
  for (int p = 0; p < 2; ++p) {
    if (h->gexec[p]) hipGraphExecDestroy(h->gexec[p]);
    if (h->graph[p]) hipGraphDestroy(h->graph[p]);
  }
  void *ptrs[] = {h->d_desc, h->d_items, h->d_patch, h->d_obs_sub, h->d_node_ij, h->d_subap_nodes,
                  h->d_obs_corner, h->d_obs_dist, h->d_bank, h->d_r, h->d_xa[0], h->d_xa[1],
                  h->d_xb, h->d_tmp, h->d_frame, h->d_flags, h->d_node_adj, h->d_slot_off,
                  h->d_slots, h->d_dom_base, h->d_ones, h->d_stats, h->d_xpbar, h->d_ybar,
                  h->d_xbbar, h->d_dbar, h->d_theta, h->d_owner_item, h->d_minv_off, h->d_minv,
                  h->d_prhs, h->d_pi, h->d_xmean, h->d_u1, h->d_u2, h->d_xprev,
                  h->d_refit, h->d_rpart, h->d_stage, h->d_smean, h->d_boff, h->d_bent,
                  h->d_bitem, h->d_bw, h->d_pterm_off, h->d_pterms, h->d_pitem, h->d_order};
  for (void *p : ptrs)
    if (p) hipFree(p);
  for (auto &e : h->tev) {
    hipEventDestroy(e.first);
    hipEventDestroy(e.second);
  }
  delete h;
}

template <typename T> void set_offsets(AnaArgsHost<T> &A, const int32_t *off) {
  A.off_xs = off[0];
  A.off_xm = off[1];
  A.off_sg = off[2];
  A.off_dd = off[3];
  A.off_yb = off[4];
  A.off_pn = off[5];
  A.off_s = off[6];
  A.off_u = off[7];
  A.off_ys = off[8];
}

template <typename T>
AnaArgsHost<T> make_args(letkf_handle *h, bool fused, const void *V, const void *y, int xa_in,
                         int xa_out) {
  AnaArgsHost<T> A;
  std::memset(&A, 0, sizeof(A));
  A.inst = h->d_desc;
  A.items = h->d_items;
  A.item_base = 0;
  A.n_items = (int32_t)h->items.size();
  A.xcd_order = h->xcd_order != LETKF_ORDER_ROW ? 1 : 0;
  A.order = h->xcd_order == LETKF_ORDER_XCD_PAIRED ? h->d_order : nullptr;
  A.noise_bank = (fused && V == nullptr) ? 1 : 0;
  A.patch_node = h->d_patch;
  A.obs_corner = h->d_obs_corner;
  A.obs_sub = h->d_obs_sub;
  A.obs_dist = h->d_obs_dist;
  A.node_ij = h->d_node_ij;
  A.r_diag = h->d_r;
  A.x_in = fused ? (const T *)h->d_xa[xa_in] : (const T *)h->d_xb;
  A.v_in = (const T *)V;
  A.bank = h->d_bank;
  A.y = (const T *)y;
  A.x_out = (T *)h->d_xa[xa_out];
  A.x_mean = h->any_piston ? (T *)h->d_xmean : nullptr;
  A.u_prev2 = h->any_loop ? (const T *)h->d_u2 : nullptr;
  A.x_prev = h->any_ar2 ? (const T *)h->d_xprev : nullptr;
  A.stage = h->any_blend ? (T *)h->d_stage : nullptr;
  A.off_clb = h->cl_off[0];
  A.off_clr = h->cl_off[1];
  A.round_items = h->round_items;
  A.p32 = h->wide_p32 ? 1 : 0;
  A.stage_mean = h->d_smean;
  A.flags = h->d_flags;
  A.frame = h->d_frame;
  A.jtol = h->jtol;
  A.max_sweeps = h->max_sweeps;
  set_offsets(A, h->fwd_off);
  return A;
}

template <typename T>
PistonArgsHost<T> make_piston_args(letkf_handle *h, const void *y, void *x) {
  PistonArgsHost<T> P;
  std::memset(&P, 0, sizeof(P));
  P.inst = h->d_desc;
  P.items = h->d_items;
  P.n_items = (int32_t)h->items.size();
  P.patch_node = h->d_patch;
  P.node_adj = h->d_node_adj;
  P.subap_nodes = h->d_subap_nodes;
  P.owner_item = h->d_owner_item;
  P.dom_base = h->d_dom_base;
  P.minv_off = h->d_minv_off;
  P.minv = h->d_minv;
  P.x_mean = (const T *)h->d_xmean;
  P.y = (const T *)y;
  P.rhs = h->d_prhs;
  P.pi = h->d_pi;
  P.x = (T *)x;
  P.term_off = h->pterm_fixed ? nullptr : h->d_pterm_off;
  P.pitem = h->d_pitem;
  P.terms = h->d_pterms;
  return P;
}

std::vector<unsigned char> piston_blob(letkf_handle *h, const void *y, void *x) {
  if (h->fp64) {
    auto P = make_piston_args<double>(h, y, x);
    return std::vector<unsigned char>((unsigned char *)&P, (unsigned char *)&P + sizeof(P));
  }
  auto P = make_piston_args<float>(h, y, x);
  return std::vector<unsigned char>((unsigned char *)&P, (unsigned char *)&P + sizeof(P));
}

// Kernels `which` in order on `s`, all with one argument block.
int launch_piston_seq(letkf_handle *h, std::initializer_list<int> which, const void *y, void *x,
                      hipStream_t s) {
  if (!h->any_piston) return LETKF_OK;
  std::vector<unsigned char> blob = piston_blob(h, y, x);
  if (blob.size() != letkf_piston_args_size(h->fp64))
    return fail(LETKF_E_DEVICE, "piston argument layout mismatch");
  for (int w : which) {
    int gx, gy;
    letkf_piston_grid(w, (int)h->items.size(), h->n_inst, h->max_nodes, h->max_elems, &gx, &gy);
    HIPCHK(letkf_launch_piston(h->fp64, w, blob.data(), gx, gy, s));
  }
  return LETKF_OK;
}

// The end of a frame after the analysis: the piston fit (right-hand sides,
// then pistons applied per domain) when enabled, and the frame counter of the
// bank draws when `frame` is given (folded into the last piston kernel); then
// the closed loop's command from the final ensemble x, and the online refit
// of the AR(1) model from x and the frame's input ensemble x_prev.
int launch_frame_tail(letkf_handle *h, const void *y, void *x, const void *x_prev, uint32_t *frame,
                      hipStream_t s) {
  if (h->any_blend) {
    HIPCHK(letkf_launch_blend(h->fp64, h->d_desc, h->d_items, (int)h->items.size(), h->d_patch, h->d_smean,
                              h->d_boff, h->d_bent, h->d_bitem, h->d_bw, h->d_dom_base, h->d_minv_off, h->d_minv,
                              h->d_prhs, h->d_pi, h->d_stage, x, h->any_piston ? nullptr : frame, h->max_nodes,
                              h->n_inst, s));
    frame = h->any_piston ? frame : nullptr;  // advanced by the blend gather
  }
  if (!h->any_piston) {
    if (frame) HIPCHK(letkf_launch_frame_advance(frame, s));
  } else {
    int rc = launch_piston_seq(h, {0}, y, x, s);
    if (rc) return rc;
    std::vector<unsigned char> blob = piston_blob(h, y, x);
    HIPCHK(letkf_launch_piston_finish(h->fp64, blob.data(), (int)h->items.size(), frame, s));
  }
  if (h->any_loop)
    HIPCHK(letkf_launch_command(h->fp64, h->d_desc, h->n_inst, h->max_nodes, x, h->d_u1, h->d_u2, s));
  if (h->any_refit)
    HIPCHK(letkf_launch_refit(h->fp64, h->d_desc, h->d_refit, x, x_prev, h->d_rpart, h->max_nodes, h->n_inst, s));
  return LETKF_OK;
}

// Slot -> item table of LETKF_ORDER_XCD_PAIRED.  Slot b goes to XCD b % 8
// as its (b / 8)-th workgroup; XCD x takes the contiguous run of items
// [x per, (x + 1) per) as in LETKF_ORDER_XCD.  Within a run of n items and R
// CUs per XCD (two workgroups fit a CU): for R < n <= 2R the workgroups
// R .. n - 1 share a CU with 0 .. n - R - 1, so the 2R - n costliest items take
// the CUs they hold alone and the others are paired costliest with cheapest;
// for longer runs the items go in order of falling cost (the dispatcher then
// hands the next item to the first CU that frees up, longest first).
std::vector<int32_t> paired_order(const letkf_handle *h) {
  const int n = (int)h->items.size(), grid = 8 * ((n + 7) / 8), per = grid / 8, R = h->round_items;
  std::vector<int32_t> tab((size_t)std::max(grid, 1), -1);
  for (int x = 0; x < 8; ++x) {
    std::vector<std::pair<double, int>> run;
    for (int i = x * per; i < std::min(n, (x + 1) * per); ++i) {
      const DomItem &it = h->items[i];
      const double m = h->desc[it.inst].m / 64.0;
      const double cost = 100.0 * m * m * m + 20.0 * m * m * (2.0 * it.n_obs / 72.0) + 15.0 * m * it.n_patch / 40.0;
      run.push_back({-cost, i});
    }
    std::stable_sort(run.begin(), run.end());  // costliest first
    const int nr = (int)run.size();
    std::vector<int> slot_item(per, -1);
    if (nr > R && nr <= 2 * R) {
      const int n2 = nr - R;  // CUs holding two
      for (int j = n2; j < R; ++j) slot_item[j] = run[j - n2].second;
      for (int j = 0; j < n2; ++j) {
        slot_item[j] = run[R - n2 + j].second;
        slot_item[j + R] = run[nr - 1 - j].second;
      }
    } else {
      for (int j = 0; j < nr; ++j) slot_item[j] = run[j].second;
    }
    for (int j = 0; j < per; ++j) tab[(size_t)8 * j + x] = slot_item[j];
  }
  return tab;
}

int grid_for(const letkf_handle *h) {
  const int n = (int)h->items.size();
  return h->xcd_order != LETKF_ORDER_ROW ? 8 * ((n + 7) / 8) : n;
}

int launch_analysis(letkf_handle *h, bool fused, const void *V, const void *y, int xa_in, int xa_out,
                    hipStream_t s) {
  if (h->fp64) {
    auto A = make_args<double>(h, fused, V, y, xa_in, xa_out);
    HIPCHK(letkf_launch_analysis(&A, 1, fused, h->transform, grid_for(h), h->lds, s));
  } else {
    auto A = make_args<float>(h, fused, V, y, xa_in, xa_out);
    HIPCHK(letkf_launch_analysis(&A, 0, fused, h->transform, grid_for(h), h->lds, s));
  }
  return LETKF_OK;
}

int check_noise(letkf_handle *h, const void *V) {
  if (!V && !h->all_bank)
    return fail(LETKF_E_INVAL, "no V given and not every instance has a noise bank");
  return LETKF_OK;
}

// Build (once per parity) or refresh the graph of the fused frame: the
// analysis, the differential-piston kernels when enabled, the frame counter.
int graph_step(letkf_handle *h, const void *V, const void *y, hipStream_t s) {
  const int p = h->cur;
  std::vector<unsigned char> args;
  if (h->fp64) {
    auto A = make_args<double>(h, true, V, y, p, 1 - p);
    args.assign((unsigned char *)&A, (unsigned char *)&A + sizeof(A));
  } else {
    auto A = make_args<float>(h, true, V, y, p, 1 - p);
    args.assign((unsigned char *)&A, (unsigned char *)&A + sizeof(A));
  }
  hipKernelNodeParams kp{};
  kp.blockDim = dim3(letkf_analysis_threads_for(h->transform));
  kp.gridDim = dim3(grid_for(h));
  kp.func = (void *)letkf_analysis_kernel(h->fp64, 1, h->transform);
  kp.sharedMemBytes = (unsigned)h->lds;
  // piston nodes: the right-hand side reads y; solve and apply do not
  std::vector<unsigned char> prhs, pfix;
  if (h->any_piston) {
    prhs = piston_blob(h, y, h->d_xa[1 - p]);
    pfix = piston_blob(h, nullptr, h->d_xa[1 - p]);
  }
  auto piston_params = [&](int which, std::vector<unsigned char> &blob, void **slot) {
    hipKernelNodeParams q{};
    int gx, gy;
    letkf_piston_grid(which, (int)h->items.size(), h->n_inst, h->max_nodes, h->max_elems, &gx, &gy);
    q.blockDim = dim3(letkf_analysis_threads());
    q.gridDim = dim3(gx, gy);
    q.func = (void *)letkf_piston_kernel(h->fp64, which);
    slot[0] = blob.data();
    q.kernelParams = slot;
    q.extra = nullptr;
    q.sharedMemBytes = 0;
    return q;
  };
  if (!h->gexec[p]) {
    h->gargs[p] = args;
    void *kargs[] = {h->gargs[p].data()};
    kp.kernelParams = kargs;
    kp.extra = nullptr;
    HIPCHK(hipGraphCreate(&h->graph[p], 0));
    HIPCHK(hipGraphAddKernelNode(&h->gnode[p], h->graph[p], nullptr, 0, &kp));
    hipGraphNode_t last = h->gnode[p];
    if (h->any_blend) {
      // blend-mode gather: alignment right-hand sides, pistons, weighted gather
      // (with the frame counter unless the piston kernels follow)
      int n_items = (int)h->items.size();
      void *xo = h->d_xa[1 - p];
      uint32_t *fr = h->any_piston ? nullptr : h->d_frame;
      const unsigned gi = (unsigned)((n_items + 3) / 4);
      void *b1[] = {&h->d_desc, &h->d_items, &n_items, &h->d_patch, &h->d_smean, &h->d_boff, &h->d_bent, &h->d_prhs};
      void *b2[] = {&h->d_desc, &h->d_items, &n_items, &h->d_dom_base, &h->d_minv_off, &h->d_minv, &h->d_prhs,
                    &h->d_pi};
      void *b3[] = {&h->d_desc, &h->d_boff, &h->d_bent, &h->d_bitem, &h->d_bw, &h->d_stage, &h->d_pi, &xo, &fr};
      const void *fn[3] = {letkf_blend_rhs_kernel(), letkf_blend_solve_kernel(), letkf_blend_gather_kernel(h->fp64)};
      void **ka[3] = {b1, b2, b3};
      const dim3 gd[3] = {dim3(gi), dim3(gi), dim3((unsigned)((h->max_nodes + 3) / 4), (unsigned)h->n_inst)};
      for (int t = 0; t < 3; ++t) {
        hipKernelNodeParams kb{};
        kb.blockDim = dim3(letkf_analysis_threads());
        kb.gridDim = gd[t];
        kb.func = (void *)fn[t];
        kb.kernelParams = ka[t];
        kb.extra = nullptr;
        kb.sharedMemBytes = 0;
        hipGraphNode_t nb;
        HIPCHK(hipGraphAddKernelNode(&nb, h->graph[p], &last, 1, &kb));
        last = nb;
      }
    }
    if (h->any_piston) {
      // piston right-hand sides, then pistons applied and the frame counter
      h->gpargs[p][0] = prhs;
      h->gpargs[p][1] = pfix;
      void *s0[1];
      hipKernelNodeParams q0 = piston_params(0, h->gpargs[p][0], s0);
      HIPCHK(hipGraphAddKernelNode(&h->gpnode[p][0], h->graph[p], &last, 1, &q0));
      hipKernelNodeParams q1{};
      void *s1[] = {h->gpargs[p][1].data(), &h->d_frame};
      q1.blockDim = dim3(letkf_analysis_threads());
      q1.gridDim = dim3((unsigned)h->items.size());
      q1.func = (void *)letkf_piston_finish_kernel(h->fp64);
      q1.kernelParams = s1;
      q1.extra = nullptr;
      q1.sharedMemBytes = 0;
      HIPCHK(hipGraphAddKernelNode(&h->gpnode[p][1], h->graph[p], &h->gpnode[p][0], 1, &q1));
      last = h->gpnode[p][1];
    } else if (!h->any_blend) {
      // the frame counter of the bank draws
      hipKernelNodeParams kp2{};
      void *a2[] = {&h->d_frame};
      kp2.blockDim = dim3(64);
      kp2.gridDim = dim3(1);
      kp2.func = (void *)letkf_frame_advance_kernel();
      kp2.kernelParams = a2;
      kp2.extra = nullptr;
      kp2.sharedMemBytes = 0;
      hipGraphNode_t adv;
      HIPCHK(hipGraphAddKernelNode(&adv, h->graph[p], &last, 1, &kp2));
      last = adv;
    }
    if (h->any_loop) {
      // the closed loop's command from this parity's analysis ensemble
      void *xo = h->d_xa[1 - p];
      void *c3[] = {&h->d_desc, &xo, &h->d_u1, &h->d_u2};
      hipKernelNodeParams kc{};
      kc.blockDim = dim3(letkf_analysis_threads());
      kc.gridDim = dim3((unsigned)((h->max_nodes + 3) / 4), (unsigned)h->n_inst);
      kc.func = (void *)letkf_command_kernel(h->fp64);
      kc.kernelParams = c3;
      kc.extra = nullptr;
      kc.sharedMemBytes = 0;
      hipGraphNode_t cmd;
      HIPCHK(hipGraphAddKernelNode(&cmd, h->graph[p], &last, 1, &kc));
      last = cmd;
    }
    if (h->any_refit) {
      // the online refit: sums over the nodes, then the model of the next frame
      void *xo = h->d_xa[1 - p], *xi = h->d_xa[p];
      int stride = letkf_refit_stride(h->max_nodes);
      void *c5[] = {&h->d_desc, &h->d_refit, &xo, &xi, &h->d_rpart, &stride};
      hipKernelNodeParams kr{};
      kr.blockDim = dim3(letkf_analysis_threads());
      kr.gridDim = dim3((unsigned)stride, (unsigned)h->n_inst);
      kr.func = (void *)letkf_refit_sums_kernel(h->fp64);
      kr.kernelParams = c5;
      kr.extra = nullptr;
      kr.sharedMemBytes = 0;
      hipGraphNode_t rs;
      HIPCHK(hipGraphAddKernelNode(&rs, h->graph[p], &last, 1, &kr));
      void *c6[] = {&h->d_desc, &h->d_refit, &h->d_rpart, &stride};
      hipKernelNodeParams kf{};
      kf.blockDim = dim3(letkf_analysis_threads());
      kf.gridDim = dim3((unsigned)h->n_inst);
      kf.func = (void *)letkf_refit_finish_kernel();
      kf.kernelParams = c6;
      kf.extra = nullptr;
      kf.sharedMemBytes = 0;
      hipGraphNode_t rf;
      HIPCHK(hipGraphAddKernelNode(&rf, h->graph[p], &rs, 1, &kf));
      last = rf;
    }
    if (h->any_ar2) {
      // AR(2): this frame's input ensemble becomes the next frame's history
      void *src = h->d_xa[p];
      int64_t ne = h->total_x;
      void *c4[] = {&src, &h->d_xprev, &ne};
      hipKernelNodeParams kq{};
      kq.blockDim = dim3(256);
      kq.gridDim = dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (ne + 255) / 256)));
      kq.func = (void *)letkf_copy_kernel(h->fp64);
      kq.kernelParams = c4;
      kq.extra = nullptr;
      kq.sharedMemBytes = 0;
      hipGraphNode_t cp;
      HIPCHK(hipGraphAddKernelNode(&cp, h->graph[p], &last, 1, &kq));
    }
    HIPCHK(hipGraphInstantiate(&h->gexec[p], h->graph[p], nullptr, nullptr, 0));
  } else {
    if (args != h->gargs[p]) {
      h->gargs[p] = args;
      void *kargs[] = {h->gargs[p].data()};
      kp.kernelParams = kargs;
      kp.extra = nullptr;
      HIPCHK(hipGraphExecKernelNodeSetParams(h->gexec[p], h->gnode[p], &kp));
    }
    if (h->any_piston && prhs != h->gpargs[p][0]) {
      h->gpargs[p][0] = prhs;
      void *s0[1];
      hipKernelNodeParams q0 = piston_params(0, h->gpargs[p][0], s0);
      HIPCHK(hipGraphExecKernelNodeSetParams(h->gexec[p], h->gpnode[p][0], &q0));
    }
  }
  HIPCHK(hipGraphLaunch(h->gexec[p], s));
  return LETKF_OK;
}

}  // namespace

static void instance_sizes(const InstGeom &g, letkf_sizes &s);

// ======================================================================== ABI
extern "C" {

const char *letkf_strerror(int code) {
  switch (code) {
    case LETKF_OK: return "ok";
    case LETKF_E_INVAL: return "invalid argument or configuration";
    case LETKF_E_NOMEM: return "out of memory";
    case LETKF_E_DEVICE: return "HIP runtime error";
    case LETKF_E_NONFINITE: return "non-finite slopes or update in at least one domain";
    case LETKF_E_NOCONV: return "eigensolve did not converge in at least one domain";
    case LETKF_E_STATE: return "call out of order";
    default: return "unknown error";
  }
}

const char *letkf_last_error(void) { return g_last_error.c_str(); }

int letkf_create(const letkf_config *cfgs, int32_t n_instances, int32_t device, letkf_handle **out) {
  if (!out) return fail(LETKF_E_INVAL, "out is NULL");
  *out = nullptr;
  if (const int bad = letkf_layout_check())
    return fail(LETKF_E_DEVICE, "kernel argument block " + std::to_string(bad) +
                                    " differs between the kernels and the host (mismatched build)");
  if (!cfgs || n_instances < 1) return fail(LETKF_E_INVAL, "need at least one instance");
  std::string err;
  for (int i = 0; i < n_instances; ++i) {
    if (validate(cfgs[i], i, err) != LETKF_OK) return fail(LETKF_E_INVAL, err);
    if (cfgs[i].precision != cfgs[0].precision)
      return fail(LETKF_E_INVAL, "all instances of a handle must share the precision");
    if (cfgs[i].transform != cfgs[0].transform)
      return fail(LETKF_E_INVAL, "all instances of a handle must share the transform");
    if (cfgs[i].localisation != cfgs[0].localisation)
      return fail(LETKF_E_INVAL, "all instances of a handle must share the localisation");
  }
  if (cfgs[0].transform != LETKF_TRANSFORM_NS64 && cfgs[0].transform != LETKF_TRANSFORM_NS32 &&
      cfgs[0].transform != LETKF_TRANSFORM_EVD && cfgs[0].transform != LETKF_TRANSFORM_NSP &&
      cfgs[0].transform != LETKF_TRANSFORM_NSP_MIXED)
    return fail(LETKF_E_INVAL, "unknown transform");
  letkf_handle *h = new letkf_handle();
  h->device = device;
  h->fp64 = cfgs[0].precision == LETKF_FP64;
  h->esize = h->fp64 ? 8 : 4;
  h->n_inst = n_instances;
  h->jtol = cfgs[0].jacobi_tol > 0 ? cfgs[0].jacobi_tol : (h->fp64 ? 1e-10 : 1e-4);
  h->max_sweeps = cfgs[0].max_sweeps > 0 ? cfgs[0].max_sweeps : 30;
  h->transform = cfgs[0].transform;
  if (h->fp64 && h->transform == LETKF_TRANSFORM_NS32) h->transform = LETKF_TRANSFORM_NS64;
  if (h->fp64 && h->transform == LETKF_TRANSFORM_NSP_MIXED) h->transform = LETKF_TRANSFORM_NSP;
  {
    // the P-form transforms carry the owned rows only: the blend-mode gather
    // (every patch row updated) runs the coupled FP64 iteration instead
    bool blend = false;
    for (int i = 0; i < n_instances; ++i) blend |= cfgs[i].gather_mode == LETKF_GATHER_BLEND;
    if (blend && (h->transform == LETKF_TRANSFORM_NSP || h->transform == LETKF_TRANSFORM_NSP_MIXED))
      h->transform = LETKF_TRANSFORM_NS64;
  }
  // covariance localisation has its own kernel (no transform)
  if (cfgs[0].localisation == LETKF_LOCALISATION_COVARIANCE) h->transform = kAnalysisCl;
  h->geom.resize(n_instances);
  std::vector<int32_t> patch, obs_sub, node_ij, subap_nodes;
  std::vector<uint32_t> obs_corner;
  std::vector<double> obs_dist;
  std::vector<float> bank;
  std::vector<double> r;
  std::vector<RefitState> refit;
  int64_t x_off = 0, y_off = 0, node_off = 0, bank_off = 0;
  int dom_total = 0;
  for (int i = 0; i < n_instances; ++i) {
    const letkf_config &c = cfgs[i];
    InstGeom &g = h->geom[i];
    int rc = plan_instance(c, g, err);
    if (rc != LETKF_OK) {
      free_handle(h);
      return fail(rc, "instance " + std::to_string(i) + ": " + err);
    }
    InstDesc d{};
    d.x_off = x_off;
    d.y_off = y_off;
    d.node_off = node_off;
    d.bank_off = c.noise_bank ? bank_off : -1;
    d.n_nodes = g.n_nodes;
    d.n_slopes = 2 * g.n_subaps;
    d.n_subaps = g.n_subaps;
    d.m = c.m;
    d.bank_screens = c.noise_bank ? c.bank_screens : 0;
    d.bank_side = c.noise_bank ? c.bank_side : 0;
    d.seed_lo = (uint32_t)(c.seed & 0xffffffffu);
    d.seed_hi = (uint32_t)(c.seed >> 32);
    d.instance = (uint32_t)i;
    d.piston = c.piston_removal ? 1 : 0;
    h->any_piston = h->any_piston || d.piston;
    d.model = c.model;
    h->any_loop = h->any_loop || d.model == LETKF_MODEL_CLOSED_LOOP;
    d.a = c.ar_coeff;
    d.a2 = c.ar2_coeff;
    h->any_ar2 = h->any_ar2 || d.a2 != 0.0;
    d.vscale = 1.0;
    d.blend = c.gather_mode == LETKF_GATHER_BLEND ? 1 : 0;
    h->any_blend = h->any_blend || d.blend;
    RefitState rs{};
    rs.f = c.refit_forgetting;
    rs.a0 = c.ar_coeff;
    rs.a_max = 0.9999;
    refit.push_back(rs);
    h->any_refit = h->any_refit || rs.f > 0.0;
    d.rho = c.rho;
    d.r_scale = c.r_scale;
    d.taper_c = c.taper_c;
    h->desc.push_back(d);
    for (int q = 0; q < 2 * g.n_subaps; ++q) {
      const double rv = c.r_diag ? c.r_diag[q] : c.r_sigma2;
      if (!(rv > 0)) {
        free_handle(h);
        return fail(LETKF_E_INVAL, "instance " + std::to_string(i) + ": noise variances must be > 0");
      }
      r.push_back(rv);
    }
    node_ij.insert(node_ij.end(), g.node_ij.begin(), g.node_ij.end());
    subap_nodes.insert(subap_nodes.end(), g.subap_nodes.begin(), g.subap_nodes.end());
    if (c.noise_bank) {
      const size_t nb = (size_t)c.bank_screens * c.bank_side * c.bank_side;
      bank.insert(bank.end(), c.noise_bank, c.noise_bank + nb);
      bank_off += (int64_t)nb;
      h->any_bank = true;
    } else {
      h->all_bank = false;
    }
    h->dom_base.push_back(dom_total);
    for (size_t dd = 0; dd < g.owned.size(); ++dd) {
      DomItem it{};
      it.inst = i;
      it.dom = (int)dd;
      it.n_own = (int)g.owned[dd].size();
      it.n_patch = (int)g.patch[dd].size();
      it.n_obs = (int)g.obs_sub[dd].size();
      it.patch_off = (int)patch.size();
      it.obs_off = (int)obs_sub.size();
      patch.insert(patch.end(), g.patch[dd].begin(), g.patch[dd].end());
      obs_sub.insert(obs_sub.end(), g.obs_sub[dd].begin(), g.obs_sub[dd].end());
      obs_corner.insert(obs_corner.end(), g.obs_corner[dd].begin(), g.obs_corner[dd].end());
      obs_dist.insert(obs_dist.end(), g.obs_dist[dd].begin(), g.obs_dist[dd].end());
      h->items.push_back(it);
      h->max_patch = std::max(h->max_patch, it.n_patch);
      h->max_obs_sub = std::max(h->max_obs_sub, it.n_obs);
      h->max_own = std::max(h->max_own, it.n_own);
      h->total_obs += 2 * it.n_obs;
    }
    dom_total += (int)g.owned.size();
    h->max_m = std::max(h->max_m, c.m);
    h->max_subaps = std::max(h->max_subaps, g.n_subaps);
    h->max_nodes = std::max(h->max_nodes, g.n_nodes);
    h->max_elems = std::max(h->max_elems, (int64_t)g.n_nodes * c.m);
    x_off += (int64_t)g.n_nodes * c.m;
    y_off += 2LL * g.n_subaps;
    node_off += g.n_nodes;
  }
  h->total_x = x_off;
  h->total_y = y_off;
  h->total_nodes = node_off;
  // LDS layout of the analysis kernel
  const size_t T = h->esize;
  const size_t p4 = (size_t)((2 * h->max_obs_sub + 3) & ~3);
  size_t o = 0;
  h->off[0] = (int32_t)o; o = align16(o + (size_t)h->max_patch * kXsStride * T);
  h->off[1] = (int32_t)o; o = align16(o + 64 * T);
  h->off[2] = (int32_t)o; o = align16(o + 2 * (size_t)h->max_obs_sub * 8);
  h->off[3] = (int32_t)o; o = align16(o + 2 * (size_t)h->max_obs_sub * 8);
  h->off[4] = (int32_t)o; o = align16(o + 2 * (size_t)h->max_obs_sub * T);
  h->off[5] = (int32_t)o; o = align16(o + 192 * 4 + 64 * 8);  // patch nodes, their (i, j), corners, u_{k-2}
  h->off[6] = (int32_t)o; o = align16(o + letkf_analysis_scratch_doubles() * 8);
  h->off[7] = (int32_t)o;
  h->off[8] = (int32_t)o;
  size_t u = std::max({p4 * kYsStride * T, (size_t)64 * kXsStride * T, letkf_analysis_xch_bytes(),
                       (size_t)64 * kYsStride * T, (size_t)64 * 65 * 8});
  {
    // The analysis: small arrays, then the patch rows, of which only the owned
    // ones (rows 0 .. n_own - 1) outlive stage 2; the others run on into the U
    // area, which holds A~ and then the two FP64 64 x 64 matrices of its inverse
    // square root from stage 3 on; the slopes operand ys of stages 2-3 sits at
    // the end of U, clear of those rows.  FP32 at 80x80, m = 64: 79.7 KB, under
    // 80 KiB: two workgroups per CU.
    size_t f = 0;
    h->fwd_off[1] = (int32_t)f; f = align16(f + 64 * T);
    h->fwd_off[2] = (int32_t)f; f = align16(f + 2 * (size_t)h->max_obs_sub * 8);
    h->fwd_off[3] = (int32_t)f; f = align16(f + 2 * (size_t)h->max_obs_sub * 8);
    h->fwd_off[4] = (int32_t)f; f = align16(f + 2 * (size_t)h->max_obs_sub * T);
    h->fwd_off[5] = (int32_t)f; f = align16(f + 192 * 4 + 64 * 8);
    // (the Jacobi transform uses the whole scratch, the Newton-Schulz ones its head)
    const size_t scratch = h->transform == LETKF_TRANSFORM_EVD ? letkf_analysis_scratch_doubles()
                                                               : letkf_analysis_fwd_scratch_doubles();
    h->fwd_off[6] = (int32_t)f; f = align16(f + scratch * 8);
    h->fwd_off[0] = (int32_t)f;
    // (blend mode updates every patch row: the rows past the owned ones are
    // staged again after the transform; the P-form transforms carry V = X' Z
    // in place of the owned rows, in whole 16-row blocks)
    const bool nsp = h->transform == LETKF_TRANSFORM_NSP || h->transform == LETKF_TRANSFORM_NSP_MIXED;
    const size_t own_rows = nsp ? (size_t)16 * ((h->max_own + 15) / 16) : (size_t)h->max_own;
    const size_t ub = align16(f + own_rows * kXsStride * T);
    const size_t rows_end = f + (size_t)h->max_patch * kXsStride * T;  // end of the patch rows
    const size_t ys_bytes = p4 * kYsStride * T;
    const size_t spill = rows_end > ub ? align16(rows_end - ub) : 0;
    // Newton-Schulz in FP64: A~, then the two FP64 iterates; with FP32
    // iterates: three of them and the FP32 Gram (row stride 68); Jacobi: A~
    // and its factor (the block exchange and W reuse the area)
    // (the P-form transforms: A~ then P, and P^2, in the two FP64 areas)
    const size_t iter_bytes = h->transform == LETKF_TRANSFORM_NS32   ? (size_t)4 * 64 * 68 * 4
                              : h->transform == LETKF_TRANSFORM_EVD ? std::max(u, (size_t)64 * 65 * 8)
                                                                    : (size_t)2 * 64 * 65 * 8;
    const size_t uf = std::max(iter_bytes, spill + ys_bytes);
    h->fwd_off[7] = (int32_t)ub;
    h->fwd_off[8] = (int32_t)(ub + uf - ys_bytes);
    h->lds = align16(ub + uf);
    if (h->transform == kAnalysisCl) {
      // covariance localisation: every patch row (read again by the update),
      // then one FP64 area for X'_P^T, P_loc and S (packed lower triangle) in
      // turn, and B with a spare row (its owned rows and one more become the
      // solve's columns); no slope operand.  FP32 at 80x80: under 80 KiB, two
      // workgroups per CU
      const size_t pmax = 2 * (size_t)h->max_obs_sub, ld = pmax + 1;
      const size_t rows = align16(f + (size_t)h->max_patch * kXsStride * T);
      const size_t sreg = std::max({(size_t)64 * 65 * 8, (size_t)64 * kClXtStride * 8, pmax * (pmax + 1) / 2 * 8});
      h->fwd_off[7] = (int32_t)rows;
      h->fwd_off[8] = (int32_t)rows;
      h->cl_off[0] = (int32_t)align16(rows + sreg);
      h->cl_off[1] = h->cl_off[0];
      h->lds = align16(h->cl_off[0] + ((size_t)h->max_patch + 1) * ld * 8);
    }
  }
  // Shapes past 64 members or past the 64-node patch run the wide analysis
  // (8 wavefronts a work item, the FP64 P-form iteration); it has the
  // delay-free AR(1) phase model with the concatenating gather only.
  h->wide = h->max_m > kLanes || h->max_patch > kMaxPatch || h->max_obs_sub > kMaxObsSub;
  if (h->wide) {
    std::string why;
    if (h->any_loop) why = "the closed-loop model";
    else if (h->any_ar2) why = "the AR(2) model";
    else if (h->any_refit) why = "the online refit";
    else if (h->any_blend) why = "the blend-mode gather";
    else if (h->transform == kAnalysisCl) why = "covariance localisation";
    else if (h->transform == LETKF_TRANSFORM_EVD || h->transform == LETKF_TRANSFORM_NS32)
      why = "the EVD and NS32 transforms (it runs the P-form iteration in FP64)";
    if (!why.empty()) {
      free_handle(h);
      return fail(LETKF_E_INVAL, "more than 64 members or a patch of more than 64 nodes runs the wide analysis, "
                                 "which has no " + why);
    }
    const int nb = std::max(4, (h->max_m + 15) / 16), M = 16 * nb;
    h->wide_p32 = !h->fp64 && h->transform == LETKF_TRANSFORM_NSP_MIXED;
    h->transform = kAnalysisWide + nb;
    // small arrays, then the patch rows (row stride M + 1); the Gram's
    // 16-slope operand after them.  From the transform on: V in place of the
    // first owned-row blocks, its second buffer and the stored upper block
    // triangle of P after them, over the dead patch rows and operand.
    const size_t T = h->esize, XS = M + 1, YS = M + 1;
    const size_t vrows = (size_t)16 * ((h->max_own + 15) / 16);
    size_t f = 0;
    h->fwd_off[5] = (int32_t)f; f = align16(f + letkf_wide_pn_ints() * 4);
    h->fwd_off[6] = (int32_t)f; f = align16(f + letkf_wide_scratch_doubles() * 8);
    h->fwd_off[1] = (int32_t)f; f = align16(f + (size_t)kMaxPatchWide * 8);
    h->fwd_off[2] = (int32_t)f; f = align16(f + 2 * (size_t)h->max_obs_sub * 8);
    h->fwd_off[3] = (int32_t)f; f = align16(f + 2 * (size_t)h->max_obs_sub * 8);
    h->fwd_off[4] = (int32_t)f; f = align16(f + 2 * (size_t)h->max_obs_sub * 8);
    h->fwd_off[0] = (int32_t)f;
    const size_t xrows = std::max((size_t)h->max_patch, vrows) * XS * T;
    h->fwd_off[8] = (int32_t)align16(f + xrows);
    const size_t end1 = h->fwd_off[8] + (size_t)16 * YS * 8;
    h->cl_off[0] = (int32_t)align16(f + vrows * XS * T);
    h->cl_off[1] = h->cl_off[0];
    h->fwd_off[7] = (int32_t)align16(h->cl_off[0] + vrows * XS * T);
    const size_t end2 = h->fwd_off[7] + letkf_wide_tri_bytes(nb);
    h->lds = align16(std::max(end1, end2));
  }
  {  // the adjoint kernel: a larger U area (FP64 64 x 64: W_bar and the DK
     // products), Q (then S) in the state's precision, scratch.  FP32 at
     // 80x80, m = 64: 78.4 KiB, so two work items share a CU
    size_t oa = align16(o + std::max(u, (size_t)64 * 65 * 8));
    h->adj_off[0] = (int32_t)oa; oa = align16(oa + (size_t)64 * 65 * T);
    h->adj_off[1] = (int32_t)oa; oa = align16(oa + letkf_adjoint_scratch_doubles() * 8);
    h->adj_lds = oa;
  }
  // adjoint maps: node -> (subaperture for corner roles a, b, c, d), the slots
  // (item, local slope) of each subaperture in item order, item ranges
  std::vector<int32_t> node_adj, slot_off, slots, dom_base(h->dom_base);
  dom_base.push_back((int32_t)h->items.size());
  {
    const int64_t total_sub = h->total_y / 2;
    std::vector<std::vector<int32_t>> lists((size_t)total_sub);
    int64_t sb = 0;
    std::vector<int64_t> sub_base;
    for (int i = 0; i < n_instances; ++i) {
      sub_base.push_back(sb);
      const InstGeom &g = h->geom[i];
      const int N = g.N;
      std::vector<int32_t> sid((size_t)N * N, -1);
      for (int q = 0; q < g.n_subaps; ++q) sid[g.subaps[2 * q] * N + g.subaps[2 * q + 1]] = q;
      for (int n = 0; n < g.n_nodes; ++n) {
        const int ni = g.node_ij[2 * n], nj = g.node_ij[2 * n + 1];
        const int si[4] = {ni, ni, ni - 1, ni - 1}, sj[4] = {nj, nj - 1, nj, nj - 1};
        for (int r = 0; r < 4; ++r) {
          int v = -1;
          if (si[r] >= 0 && si[r] < N && sj[r] >= 0 && sj[r] < N && sid[si[r] * N + sj[r]] >= 0)
            v = (int32_t)(sb + sid[si[r] * N + sj[r]]);
          node_adj.push_back(v);
        }
      }
      sb += g.n_subaps;
    }
    // pairs (x slot, n_obs): the y slope of a slot sits n_obs slots later
    for (const DomItem &it : h->items) {
      const InstGeom &g = h->geom[it.inst];
      for (int o = 0; o < it.n_obs; ++o) {
        auto &l = lists[(size_t)(sub_base[it.inst] + g.obs_sub[it.dom][o])];
        l.push_back(2 * it.obs_off + o);
        l.push_back(it.n_obs);
      }
    }
    slot_off.push_back(0);
    for (int64_t k = 0; k < total_sub; ++k) {
      slots.insert(slots.end(), lists[(size_t)k].begin(), lists[(size_t)k].end());
      slot_off.push_back((int32_t)(slots.size() / 2));
    }
  }

  // differential pistons: owning item of every node, M^+ per instance
  std::vector<int32_t> owner_item((size_t)std::max<int64_t>(h->total_nodes, 1), 0);
  std::vector<int64_t> minv_off;
  std::vector<double> minv;
  for (size_t k = 0; k < h->items.size(); ++k) {
    const DomItem &it = h->items[k];
    const InstGeom &g = h->geom[it.inst];
    for (int32_t nd_ : g.owned[it.dom]) owner_item[(size_t)(h->desc[it.inst].node_off + nd_)] = (int32_t)k;
  }
  for (int i = 0; i < n_instances; ++i) {
    minv_off.push_back((int64_t)minv.size());
    if (!h->desc[i].piston && !h->desc[i].blend) continue;
    std::vector<double> mi;
    if ((h->desc[i].piston ? piston_minv(h->geom[i], mi, err) : blend_minv(h->geom[i], mi, err)) != LETKF_OK) {
      free_handle(h);
      return fail(LETKF_E_INVAL, "instance " + std::to_string(i) + ": " + err);
    }
    minv.insert(minv.end(), mi.begin(), mi.end());
  }
  std::vector<PistonItem> pitem(std::max<size_t>(h->items.size(), 1), PistonItem{});
  for (size_t k = 0; k < h->items.size(); ++k) {
    const DomItem &it = h->items[k];
    const InstDesc &ds = h->desc[(size_t)it.inst];
    PistonItem &pr = pitem[k];
    pr.b0 = h->dom_base[(size_t)it.inst];
    pr.nd = (int32_t)h->geom[(size_t)it.inst].owned.size();
    pr.row = minv_off[(size_t)it.inst] + (int64_t)(k - (size_t)pr.b0) * pr.nd;
    pr.x_off = ds.x_off;
    pr.patch_off = it.patch_off;
    pr.n_own = it.n_own;
    pr.m = ds.m;
    pr.piston = ds.piston ? 1 : 0;
  }

  // piston right-hand sides: per item, the subapertures its domain shares
  // with others and the summed coefficients of its own corners
  std::vector<int32_t> pterm_off(1, 0);
  std::vector<PistonTerm> pterms;
  for (int i = 0; i < n_instances; ++i) {
    const InstGeom &g = h->geom[i];
    const int nd = (int)g.owned.size();
    std::vector<std::vector<PistonTerm>> per((size_t)nd);
    if (h->desc[i].piston) {
      for (int qs = 0; qs < g.n_subaps; ++qs) {
        const int32_t *cn = &g.subap_nodes[4 * qs];
        int dl[4], n = 0;
        float cx[4], cy[4];
        for (int t = 0; t < 4; ++t) {
          const int d = g.owner[cn[t]];
          int k = 0;
          while (k < n && dl[k] != d) ++k;
          if (k == n) {
            dl[n] = d;
            cx[n] = cy[n] = 0.0f;
            ++n;
          }
          cx[k] += (t & 1) ? 0.5f : -0.5f;
          cy[k] += (t & 2) ? 0.5f : -0.5f;
        }
        if (n < 2) continue;  // inside one domain: the coefficients sum to zero
        for (int k = 0; k < n; ++k) {
          if (cx[k] == 0.0f && cy[k] == 0.0f) continue;
          PistonTerm pt;
          for (int t = 0; t < 4; ++t) pt.c[t] = (int32_t)(h->desc[i].node_off + cn[t]);
          pt.yx = (int32_t)(h->desc[i].y_off + qs);
          pt.yy = (int32_t)(h->desc[i].y_off + g.n_subaps + qs);
          pt.cx = cx[k];
          pt.cy = cy[k];
          per[(size_t)dl[k]].push_back(pt);
        }
      }
    }
    for (int d = 0; d < nd; ++d) {
      pterms.insert(pterms.end(), per[(size_t)d].begin(), per[(size_t)d].end());
      pterm_off.push_back((int32_t)pterms.size());
    }
  }
  // at most 64 terms an item: the same terms at a fixed stride of 64 (one
  // load fewer before the means), the rest with coefficients 0 at node 0
  h->pterm_fixed = true;
  for (size_t k = 0; k + 1 < pterm_off.size(); ++k)
    if (pterm_off[k + 1] - pterm_off[k] > 64) h->pterm_fixed = false;
  if (h->pterm_fixed) {
    PistonTerm none{};
    for (int t = 0; t < 4; ++t) none.c[t] = 0;
    none.yx = none.yy = 0;
    none.cx = none.cy = 0.0f;
    std::vector<PistonTerm> fixed(std::max<size_t>(h->items.size(), 1) * 64, none);
    for (size_t k = 0; k + 1 < pterm_off.size(); ++k)
      for (int t = pterm_off[k]; t < pterm_off[k + 1]; ++t) fixed[k * 64 + (size_t)(t - pterm_off[k])] = pterms[(size_t)t];
    pterms.swap(fixed);
  }

  // blend-mode gather: per node of a blend instance, its patch entries (item
  // order), their items and normalised tent weights
  std::vector<int32_t> boff(1, 0), bent, bitem;
  std::vector<double> bw;
  if (h->any_blend) {
    std::vector<std::vector<std::pair<int32_t, double>>> lists((size_t)h->total_nodes);
    std::vector<int32_t> ent_item;
    for (size_t k = 0; k < h->items.size(); ++k) {
      const DomItem &it = h->items[k];
      if (!h->desc[it.inst].blend) continue;
      const InstGeom &g = h->geom[it.inst];
      const auto &P = g.patch[it.dom];
      for (size_t r = 0; r < P.size(); ++r)
        lists[(size_t)(h->desc[it.inst].node_off + P[r])].push_back(
            {(int32_t)(it.patch_off + r), blend_weight(g, it.dom, P[r])});
    }
    std::vector<int32_t> item_of(patch.size(), 0);
    for (size_t k = 0; k < h->items.size(); ++k)
      for (int r = 0; r < h->items[k].n_patch; ++r) item_of[(size_t)h->items[k].patch_off + r] = (int32_t)k;
    for (const auto &lst : lists) {
      double sw = 0.0;
      for (const auto &e : lst) sw += e.second;
      for (const auto &e : lst) {
        bent.push_back(e.first);
        bitem.push_back(item_of[(size_t)e.first]);
        bw.push_back(e.second / sw);
      }
      boff.push_back((int32_t)bent.size());
    }
  }

  int rc = LETKF_OK;
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) {
    free_handle(h);
    return fail(LETKF_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
  }
  {
    int max_lds = 0;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess &&
        h->lds > (size_t)max_lds) {
      const std::string msg = "the analysis needs " + std::to_string(h->lds) + " bytes of LDS, the device gives " +
                              std::to_string(max_lds) + " (smaller domains or halo)";
      free_handle(h);
      return fail(LETKF_E_INVAL, msg);
    }
  }
  {
    // one dispatch round of workgroups per XCD: its CUs (eight XCDs)
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && n_cu >= 8)
      h->round_items = n_cu / 8;
  }
  for (int fused = 0; fused < 2; ++fused)
    hipFuncSetAttribute(letkf_analysis_kernel(h->fp64, fused, h->transform),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)h->lds);
  {
    int max_lds = 0;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess &&
        h->adj_lds <= (size_t)max_lds) {
      h->adj_ok = hipFuncSetAttribute(letkf_adjoint_kernel(h->fp64),
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)h->adj_lds) == hipSuccess;
    }
  }
  (void)hipGetLastError();
  if ((rc = to_device(&h->d_desc, h->desc)) || (rc = to_device(&h->d_items, h->items)) ||
      (h->any_refit && (rc = to_device(&h->d_refit, refit))) ||
      (h->any_refit &&
       (rc = to_device(&h->d_rpart, std::vector<double>((size_t)n_instances * letkf_refit_stride(h->max_nodes) * 4,
                                                        0.0)))) ||
      (rc = to_device(&h->d_patch, patch)) || (rc = to_device(&h->d_obs_sub, obs_sub)) ||
      (rc = to_device(&h->d_obs_corner, obs_corner)) || (rc = to_device(&h->d_obs_dist, obs_dist)) ||
      (rc = to_device(&h->d_node_ij, node_ij)) || (rc = to_device(&h->d_subap_nodes, subap_nodes)) ||
      (rc = to_device(&h->d_r, r)) || (rc = to_device(&h->d_bank, bank)) ||
      (rc = to_device(&h->d_node_adj, node_adj)) || (rc = to_device(&h->d_slot_off, slot_off)) ||
      (rc = to_device(&h->d_slots, slots)) || (rc = to_device(&h->d_dom_base, dom_base)) ||
      (rc = to_device(&h->d_ones, std::vector<double>((size_t)n_instances, 1.0))) ||
      (rc = to_device(&h->d_stats, std::vector<double>(letkf_resvar_stats_doubles(n_instances), 0.0))) ||
      (rc = to_device(&h->d_owner_item, owner_item)) || (rc = to_device(&h->d_minv_off, minv_off)) ||
      (rc = to_device(&h->d_minv, minv)) ||
      (rc = to_device(&h->d_prhs, std::vector<double>(std::max<size_t>(h->items.size(), 1), 0.0))) ||
      (rc = to_device(&h->d_pi, std::vector<double>(std::max<size_t>(h->items.size(), 1), 0.0))) ||
      (rc = to_device(&h->d_pterm_off, pterm_off)) || (rc = to_device(&h->d_pterms, pterms)) ||
      (rc = to_device(&h->d_pitem, pitem)) || (rc = to_device(&h->d_order, paired_order(h))) ||
      (h->any_blend && ((rc = to_device(&h->d_boff, boff)) || (rc = to_device(&h->d_bent, bent)) ||
                        (rc = to_device(&h->d_bitem, bitem)) || (rc = to_device(&h->d_bw, bw)) ||
                        (rc = to_device(&h->d_smean, std::vector<double>(patch.size(), 0.0)))))) {
    free_handle(h);
    return rc;
  }
  const size_t xbytes = (size_t)h->total_x * T;
  for (void **p : {&h->d_xa[0], &h->d_xa[1], &h->d_xb}) {
    if (hipMalloc(p, std::max<size_t>(xbytes, 16)) != hipSuccess) {
      free_handle(h);
      return fail(LETKF_E_NOMEM, "hipMalloc of the ensemble failed");
    }
    hipMemset(*p, 0, std::max<size_t>(xbytes, 16));
  }
  if (hipMalloc(&h->d_tmp, std::max<size_t>((size_t)h->total_nodes * T, 16)) != hipSuccess ||
      hipMalloc(&h->d_xmean, std::max<size_t>((size_t)h->total_nodes * T, 16)) != hipSuccess ||
      hipMalloc((void **)&h->d_frame, 16) != hipSuccess ||
      hipMalloc((void **)&h->d_flags, std::max<size_t>(h->items.size(), 1) * 4) != hipSuccess) {
    free_handle(h);
    return fail(LETKF_E_NOMEM, "hipMalloc failed");
  }
  hipMemset(h->d_frame, 0, 16);
  hipMemset(h->d_flags, 0, std::max<size_t>(h->items.size(), 1) * 4);
  if (h->any_blend) {
    const size_t sb = std::max<size_t>(patch.size() * 64 * T, 16);
    if (hipMalloc(&h->d_stage, sb) != hipSuccess) {
      free_handle(h);
      return fail(LETKF_E_NOMEM, "hipMalloc of the blend staging rows failed");
    }
    hipMemset(h->d_stage, 0, sb);
  }
  if (h->any_ar2 || h->any_refit) {
    if (hipMalloc(&h->d_xprev, std::max<size_t>(xbytes, 16)) != hipSuccess) {
      free_handle(h);
      return fail(LETKF_E_NOMEM, "hipMalloc of the previous analysis ensemble failed");
    }
    hipMemset(h->d_xprev, 0, std::max<size_t>(xbytes, 16));
  }
  if (h->any_loop) {
    const size_t ub = std::max<size_t>((size_t)h->total_nodes * T, 16);
    if (hipMalloc(&h->d_u1, ub) != hipSuccess || hipMalloc(&h->d_u2, ub) != hipSuccess) {
      free_handle(h);
      return fail(LETKF_E_NOMEM, "hipMalloc of the command history failed");
    }
    hipMemset(h->d_u1, 0, ub);
    hipMemset(h->d_u2, 0, ub);
  }
  e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_handle(h);
    return fail(LETKF_E_DEVICE, std::string("create: ") + hipGetErrorString(e));
  }
  *out = h;
  return LETKF_OK;
}

void letkf_destroy(letkf_handle *h) { free_handle(h); }

int letkf_query(letkf_handle *h, int32_t instance, letkf_sizes *out) {
  if (!h || !out) return fail(LETKF_E_INVAL, "NULL argument");
  if (instance < -1 || instance >= h->n_inst) return fail(LETKF_E_INVAL, "bad instance");
  letkf_sizes s{};
  s.n_instances = h->n_inst;
  if (instance < 0) {
    s.n_nodes = h->total_nodes;
    s.n_slopes = h->total_y;
    s.n_domains = (int64_t)h->items.size();
    s.ensemble_elems = h->total_x;
    s.obs_total = h->total_obs;
    s.m = h->max_m;
    s.max_owned = h->max_own;
    s.max_obs = 2 * h->max_obs_sub;
    s.max_patch = h->max_patch;
  } else {
    instance_sizes(h->geom[instance], s);
    s.n_instances = h->n_inst;
  }
  *out = s;
  return LETKF_OK;
}

static void export_maps(const InstGeom &g, int32_t *node_ij, int32_t *owner, int32_t *obs_off,
                        int32_t *obs_idx, int32_t *own_off, int32_t *own_idx) {
  if (node_ij) std::copy(g.node_ij.begin(), g.node_ij.end(), node_ij);
  if (owner) std::copy(g.owner.begin(), g.owner.end(), owner);
  const int nd = (int)g.owned.size();
  int64_t o = 0, w = 0;
  for (int d = 0; d < nd; ++d) {
    if (obs_off) obs_off[d] = (int32_t)o;
    if (own_off) own_off[d] = (int32_t)w;
    for (int q : g.obs_sub[d]) {
      if (obs_idx) obs_idx[o] = q;
      ++o;
    }
    for (int q : g.obs_sub[d]) {
      if (obs_idx) obs_idx[o] = q + g.n_subaps;
      ++o;
    }
    for (int n : g.owned[d]) {
      if (own_idx) own_idx[w] = n;
      ++w;
    }
  }
  if (obs_off) obs_off[nd] = (int32_t)o;
  if (own_off) own_off[nd] = (int32_t)w;
}

static void instance_sizes(const InstGeom &g, letkf_sizes &s) {
  s = letkf_sizes{};
  s.n_instances = 1;
  s.n_nodes = g.n_nodes;
  s.n_slopes = 2 * g.n_subaps;
  s.n_domains = (int64_t)g.owned.size();
  s.ensemble_elems = (int64_t)g.n_nodes * g.m;
  s.m = g.m;
  s.n_sub = g.N;
  for (size_t d = 0; d < g.owned.size(); ++d) {
    s.obs_total += 2 * (int64_t)g.obs_sub[d].size();
    s.max_owned = std::max(s.max_owned, (int32_t)g.owned[d].size());
    s.max_obs = std::max(s.max_obs, (int32_t)(2 * g.obs_sub[d].size()));
    s.max_patch = std::max(s.max_patch, (int32_t)g.patch[d].size());
  }
}

int letkf_geometry(letkf_handle *h, int32_t instance, int32_t *node_ij, int32_t *owner,
                   int32_t *obs_off, int32_t *obs_idx, int32_t *own_off, int32_t *own_idx) {
  if (!h || instance < 0 || instance >= h->n_inst) return fail(LETKF_E_INVAL, "bad instance");
  export_maps(h->geom[instance], node_ij, owner, obs_off, obs_idx, own_off, own_idx);
  return LETKF_OK;
}

int letkf_plan(const letkf_config *cfg, letkf_sizes *sizes, int32_t *node_ij, int32_t *owner,
               int32_t *obs_off, int32_t *obs_idx, int32_t *own_off, int32_t *own_idx) {
  if (!cfg) return fail(LETKF_E_INVAL, "cfg is NULL");
  std::string err;
  if (validate(*cfg, 0, err) != LETKF_OK) return fail(LETKF_E_INVAL, err);
  InstGeom g;
  if (plan_instance(*cfg, g, err) != LETKF_OK) return fail(LETKF_E_INVAL, err);
  if (sizes) instance_sizes(g, *sizes);
  export_maps(g, node_ij, owner, obs_off, obs_idx, own_off, own_idx);
  return LETKF_OK;
}

int letkf_forecast(letkf_handle *h, const void *V_dev, void *stream) {
  if (!h) return fail(LETKF_E_INVAL, "NULL handle");
  int rc = check_noise(h, V_dev);
  if (rc) return rc;
  hipSetDevice(h->device);
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(letkf_launch_forecast(h->fp64, h->d_desc, h->n_inst, h->d_node_ij, h->d_xa[h->cur], V_dev,
                               h->d_bank, h->d_frame, h->d_xb, h->d_xprev, h->max_elems, s));
  HIPCHK(letkf_launch_frame_advance(h->d_frame, s));
  // AR(2), refit: X_a(k-1) becomes the history before the analysis overwrites it
  if (h->any_ar2 || h->any_refit) HIPCHK(letkf_launch_copy(h->fp64, h->d_xa[h->cur], h->d_xprev, h->total_x, s));
  h->have_xb = true;
  return LETKF_OK;
}

int letkf_analyse(letkf_handle *h, const void *y_dev, void *stream) {
  if (!h || !y_dev) return fail(LETKF_E_INVAL, "NULL argument");
  if (!h->have_xb) return fail(LETKF_E_STATE, "letkf_analyse needs a preceding letkf_forecast");
  hipSetDevice(h->device);
  int rc = launch_analysis(h, false, nullptr, y_dev, h->cur, h->cur, (hipStream_t)stream);
  if (rc) return rc;
  if ((rc = launch_frame_tail(h, y_dev, h->d_xa[h->cur], h->d_xprev, nullptr, (hipStream_t)stream))) return rc;
  h->have_xb = false;
  return LETKF_OK;
}

int letkf_step(letkf_handle *h, const void *V_dev, const void *y_dev, void *stream) {
  if (!h || !y_dev) return fail(LETKF_E_INVAL, "NULL argument");
  int rc = check_noise(h, V_dev);
  if (rc) return rc;
  hipSetDevice(h->device);
  hipStream_t s = (hipStream_t)stream;
  if (h->use_graph) {
    rc = graph_step(h, V_dev, y_dev, s);  // analysis + frame advance
    if (rc) return rc;
  } else {
    std::pair<hipEvent_t, hipEvent_t> *ev = nullptr;
    if (h->timing) {
      if (h->tev_used == h->tev.size()) {
        std::pair<hipEvent_t, hipEvent_t> e;
        HIPCHK(hipEventCreate(&e.first));
        HIPCHK(hipEventCreate(&e.second));
        h->tev.push_back(e);
      }
      ev = &h->tev[h->tev_used++];
      HIPCHK(hipEventRecord(ev->first, s));
    }
    rc = launch_analysis(h, true, V_dev, y_dev, h->cur, 1 - h->cur, s);
    if (rc) return rc;
    if (ev) HIPCHK(hipEventRecord(ev->second, s));
    if ((rc = launch_frame_tail(h, y_dev, h->d_xa[1 - h->cur], h->d_xa[h->cur], h->d_frame, s))) return rc;
    if (h->any_ar2) HIPCHK(letkf_launch_copy(h->fp64, h->d_xa[h->cur], h->d_xprev, h->total_x, s));
  }
  h->cur = 1 - h->cur;
  h->have_xb = false;
  return LETKF_OK;
}

int letkf_step_plain(letkf_handle *h, const void *V_dev, const void *y_dev, void *stream) {
  if (!h || !y_dev) return fail(LETKF_E_INVAL, "NULL argument");
  int rc = check_noise(h, V_dev);
  if (rc) return rc;
  hipSetDevice(h->device);
  hipStream_t s = (hipStream_t)stream;
  const int n = (int)h->items.size();
  for (int i = 0; i < n; ++i) {
    if (h->fp64) {
      auto A = make_args<double>(h, true, V_dev, y_dev, h->cur, 1 - h->cur);
      A.item_base = i;
      A.xcd_order = 0;
      A.order = nullptr;
      HIPCHK(letkf_launch_analysis(&A, 1, 1, h->transform, 1, h->lds, s));
    } else {
      auto A = make_args<float>(h, true, V_dev, y_dev, h->cur, 1 - h->cur);
      A.item_base = i;
      A.xcd_order = 0;
      A.order = nullptr;
      HIPCHK(letkf_launch_analysis(&A, 0, 1, h->transform, 1, h->lds, s));
    }
  }
  if ((rc = launch_frame_tail(h, y_dev, h->d_xa[1 - h->cur], h->d_xa[h->cur], h->d_frame, s))) return rc;
  if (h->any_ar2) HIPCHK(letkf_launch_copy(h->fp64, h->d_xa[h->cur], h->d_xprev, h->total_x, s));
  h->cur = 1 - h->cur;
  h->have_xb = false;
  return LETKF_OK;
}

static int copy_state(letkf_handle *h, void *dst, const void *src, size_t bytes, int on_device,
                      bool to_dev_state) {
  hipSetDevice(h->device);
  HIPCHK(hipDeviceSynchronize());
  hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice
                              : (to_dev_state ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost);
  HIPCHK(hipMemcpy(dst, src, bytes, k));
  return LETKF_OK;
}

int letkf_get_ensemble(letkf_handle *h, void *dst, int on_device) {
  if (!h || !dst) return fail(LETKF_E_INVAL, "NULL argument");
  return copy_state(h, dst, h->d_xa[h->cur], (size_t)h->total_x * h->esize, on_device, false);
}

int letkf_set_ensemble(letkf_handle *h, const void *src, int on_device) {
  if (!h || !src) return fail(LETKF_E_INVAL, "NULL argument");
  h->have_xb = false;
  const size_t b = (size_t)h->total_x * h->esize;
  int rc = copy_state(h, h->d_xa[h->cur], src, b, on_device, true);
  if (rc || !h->any_ar2) return rc;
  return copy_state(h, h->d_xprev, src, b, on_device, true);  // the AR(2) history starts steady
}

int letkf_get_forecast(letkf_handle *h, void *dst, int on_device) {
  if (!h || !dst) return fail(LETKF_E_INVAL, "NULL argument");
  if (!h->have_xb) return fail(LETKF_E_STATE, "no forecast pending");
  return copy_state(h, dst, h->d_xb, (size_t)h->total_x * h->esize, on_device, false);
}

int letkf_get_mean(letkf_handle *h, void *dst, int on_device) {
  if (!h || !dst) return fail(LETKF_E_INVAL, "NULL argument");
  hipSetDevice(h->device);
  HIPCHK(letkf_launch_mean(h->fp64, h->d_desc, h->n_inst, h->d_xa[h->cur], h->d_tmp, h->max_nodes,
                           nullptr));
  return copy_state(h, dst, h->d_tmp, (size_t)h->total_nodes * h->esize, on_device, false);
}

int letkf_get_command(letkf_handle *h, void *dst, int on_device) {
  if (!h || !dst) return fail(LETKF_E_INVAL, "NULL argument");
  if (!h->any_loop) return fail(LETKF_E_STATE, "no instance runs the closed-loop model");
  return copy_state(h, dst, h->d_u1, (size_t)h->total_nodes * h->esize, on_device, false);
}

int letkf_set_command(letkf_handle *h, const void *u1, const void *u2, int on_device) {
  if (!h || !u1 || !u2) return fail(LETKF_E_INVAL, "NULL argument");
  if (!h->any_loop) return fail(LETKF_E_STATE, "no instance runs the closed-loop model");
  const size_t b = (size_t)h->total_nodes * h->esize;
  int rc = copy_state(h, h->d_u1, u1, b, on_device, true);
  return rc ? rc : copy_state(h, h->d_u2, u2, b, on_device, true);
}

int letkf_get_frame(letkf_handle *h, uint32_t *frame) {
  if (!h || !frame) return fail(LETKF_E_INVAL, "NULL argument");
  return copy_state(h, frame, h->d_frame, 4, 0, false);
}

int letkf_set_frame(letkf_handle *h, uint32_t frame) {
  if (!h) return fail(LETKF_E_INVAL, "NULL handle");
  return copy_state(h, h->d_frame, &frame, 4, 0, true);
}

int letkf_status(letkf_handle *h, int32_t *flags) {
  if (!h || !flags) return fail(LETKF_E_INVAL, "NULL argument");
  std::vector<int32_t> f(h->items.size());
  int rc = copy_state(h, f.data(), h->d_flags, f.size() * 4, 0, false);
  if (rc) return rc;
  int any = 0;
  for (size_t i = 0; i < f.size(); ++i) {
    const DomItem &it = h->items[i];
    flags[h->dom_base[it.inst] + it.dom] = f[i];
    any |= f[i];
  }
  if (any & LETKF_FLAG_NONFINITE) return LETKF_E_NONFINITE;
  if (any & LETKF_FLAG_NOCONV) return LETKF_E_NOCONV;
  return LETKF_OK;
}

int letkf_set_params(letkf_handle *h, int32_t instance, double rho, double r_scale, double taper_c) {
  if (!h || instance < 0 || instance >= h->n_inst) return fail(LETKF_E_INVAL, "bad instance");
  if (!(rho > 0) || !(r_scale > 0) || !(taper_c >= 0)) return fail(LETKF_E_INVAL, "bad parameter");
  InstDesc &d = h->desc[instance];
  d.rho = rho;
  d.r_scale = r_scale;
  d.taper_c = taper_c;
  hipSetDevice(h->device);
  HIPCHK(hipDeviceSynchronize());
  // the device copy may hold a refitted model (a, noise scale): keep it
  InstDesc dv;
  HIPCHK(hipMemcpy(&dv, h->d_desc + instance, sizeof(dv), hipMemcpyDeviceToHost));
  dv.rho = rho;
  dv.r_scale = r_scale;
  dv.taper_c = taper_c;
  HIPCHK(hipMemcpy(h->d_desc + instance, &dv, sizeof(dv), hipMemcpyHostToDevice));
  return LETKF_OK;
}

int letkf_get_model(letkf_handle *h, double *a, double *noise_scale) {
  if (!h || (!a && !noise_scale)) return fail(LETKF_E_INVAL, "NULL argument");
  std::vector<InstDesc> dv(h->n_inst);
  int rc = copy_state(h, dv.data(), h->d_desc, dv.size() * sizeof(InstDesc), 0, false);
  if (rc) return rc;
  for (int i = 0; i < h->n_inst; ++i) {
    if (a) a[i] = dv[i].a;
    if (noise_scale) noise_scale[i] = dv[i].vscale;
  }
  return LETKF_OK;
}

int letkf_reset_refit(letkf_handle *h) {
  if (!h) return fail(LETKF_E_INVAL, "NULL handle");
  if (!h->any_refit) return fail(LETKF_E_STATE, "no instance refits its model");
  std::vector<RefitState> rs(h->n_inst);
  int rc = copy_state(h, rs.data(), h->d_refit, rs.size() * sizeof(RefitState), 0, false);
  if (rc) return rc;
  std::vector<InstDesc> dv(h->n_inst);
  if ((rc = copy_state(h, dv.data(), h->d_desc, dv.size() * sizeof(InstDesc), 0, false))) return rc;
  for (int i = 0; i < h->n_inst; ++i) {
    if (rs[i].f == 0.0) continue;
    rs[i].s01 = rs[i].s11 = 0.0;
    rs[i].frames = 0;
    dv[i].a = rs[i].a0;
    dv[i].vscale = 1.0;
  }
  if ((rc = copy_state(h, h->d_refit, rs.data(), rs.size() * sizeof(RefitState), 0, true))) return rc;
  return copy_state(h, h->d_desc, dv.data(), dv.size() * sizeof(InstDesc), 0, true);
}

int letkf_slopes(letkf_handle *h, const void *phase_dev, void *slopes_dev, void *stream) {
  if (!h || !phase_dev || !slopes_dev) return fail(LETKF_E_INVAL, "NULL argument");
  hipSetDevice(h->device);
  HIPCHK(letkf_launch_slopes(h->fp64, h->d_desc, h->n_inst, h->d_subap_nodes, phase_dev, slopes_dev,
                             h->max_subaps, (hipStream_t)stream));
  return LETKF_OK;
}

int letkf_set_schedule(letkf_handle *h, int32_t use_graph, int32_t order) {
  if (!h) return fail(LETKF_E_INVAL, "NULL handle");
  if (order < LETKF_ORDER_ROW || order > LETKF_ORDER_XCD_PAIRED) return fail(LETKF_E_INVAL, "unknown item order");
  if (order != h->xcd_order) {
    for (int p = 0; p < 2; ++p) {
      if (h->gexec[p]) hipGraphExecDestroy(h->gexec[p]);
      if (h->graph[p]) hipGraphDestroy(h->graph[p]);
      h->gexec[p] = nullptr;
      h->graph[p] = nullptr;
      h->gargs[p].clear();
    }
  }
  h->use_graph = use_graph ? 1 : 0;
  h->xcd_order = order;
  return LETKF_OK;
}

int letkf_get_schedule(letkf_handle *h, int32_t *use_graph, int32_t *order) {
  if (!h) return fail(LETKF_E_INVAL, "NULL handle");
  if (use_graph) *use_graph = h->use_graph;
  if (order) *order = h->xcd_order;
  return LETKF_OK;
}

extern "C++" {
namespace {
// Saves the filter state that tuning frames change and puts it back (and the
// schedule and the events) when it goes out of scope, whatever the exit path.
struct TuneGuard {
  letkf_handle *h;
  std::vector<std::pair<void *, size_t>> keep;
  std::vector<std::vector<unsigned char>> saved;
  int cur0, graph0, order0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool armed = false;
  explicit TuneGuard(letkf_handle *hh) : h(hh), cur0(hh->cur), graph0(hh->use_graph), order0(hh->xcd_order) {}
  int save() {
    const size_t xbytes = (size_t)h->total_x * h->esize, ubytes = (size_t)h->total_nodes * h->esize;
    keep = {{h->d_xa[h->cur], xbytes}, {h->d_frame, 4}, {h->d_desc, h->n_inst * sizeof(InstDesc)}};
    if (h->d_xprev) keep.push_back({h->d_xprev, xbytes});
    if (h->any_loop) {
      keep.push_back({h->d_u1, ubytes});
      keep.push_back({h->d_u2, ubytes});
    }
    if (h->any_refit) keep.push_back({h->d_refit, h->n_inst * sizeof(RefitState)});
    saved.assign(keep.size(), {});
    HIPCHK(hipDeviceSynchronize());
    for (size_t i = 0; i < keep.size(); ++i) {
      saved[i].resize(keep[i].second);
      HIPCHK(hipMemcpy(saved[i].data(), keep[i].first, keep[i].second, hipMemcpyDeviceToHost));
    }
    armed = true;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    return LETKF_OK;
  }
  ~TuneGuard() {
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (!armed) return;
    hipDeviceSynchronize();
    h->cur = cur0;
    for (size_t i = 0; i < keep.size(); ++i)
      hipMemcpy(keep[i].first, saved[i].data(), keep[i].second, hipMemcpyHostToDevice);
    (void)hipGetLastError();
  }
};
}  // namespace
}  // extern "C++"

int letkf_autotune(letkf_handle *h, const void *V_dev, const void *y_dev, int32_t frames,
                   const char *cache_path, void *stream) {
  if (!h || !y_dev || frames < 1) return fail(LETKF_E_INVAL, "bad argument");
  int dev_cu = 0;
  hipDeviceGetAttribute(&dev_cu, hipDeviceAttributeMultiprocessorCount, h->device);
  std::ostringstream key;
  int ar2 = h->any_ar2 ? 1 : 0, refit = h->any_refit ? 1 : 0;
  const int loc = h->transform == kAnalysisCl ? 1 : 0;  // the transform field names CL's own kernel
  int model = 0, gather = 0;
  for (const auto &d : h->desc) {
    model |= d.model;
    gather |= d.blend;
  }
  key << "gfx950 cu " << dev_cu << " fp" << (h->fp64 ? 64 : 32) << " items " << h->items.size() << " m "
      << h->max_m << " patch " << h->max_patch << " obs " << h->max_obs_sub << " transform " << h->transform
      << (h->wide_p32 ? " p32" : "") << " localisation " << loc << " model " << model << " gather " << gather << " ar2 " << ar2
      << " refit " << refit;
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      const size_t bar = line.find(" | ");
      if (bar != std::string::npos && line.substr(0, bar) == key.str()) {
        int g = 1, x = 1;
        if (sscanf(line.c_str() + bar + 3, "graph %d order %d", &g, &x) == 2)
          return letkf_set_schedule(h, g, x);
      }
    }
  }
  hipStream_t s = (hipStream_t)stream;
  hipSetDevice(h->device);
  // tuning frames must not change the filter state: the guard restores it on
  // every return below
  TuneGuard guard(h);
  int rc = guard.save();
  if (rc) return rc;
  float best = 1e30f;
  int bg = 1, bx = LETKF_ORDER_XCD;
  for (int g = 0; g < 2; ++g)
    for (int x = LETKF_ORDER_ROW; x <= LETKF_ORDER_XCD_PAIRED; ++x) {
      if ((rc = letkf_set_schedule(h, g, x))) return rc;
      if ((rc = letkf_step(h, V_dev, y_dev, stream))) return rc;  // warm-up (and graph build)
      HIPCHK(hipEventRecord(guard.e0, s));
      for (int f = 0; f < frames; ++f)
        if ((rc = letkf_step(h, V_dev, y_dev, stream))) return rc;
      HIPCHK(hipEventRecord(guard.e1, s));
      HIPCHK(hipEventSynchronize(guard.e1));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, guard.e0, guard.e1));
      if (ms < best) {
        best = ms;
        bg = g;
        bx = x;
      }
    }
  if ((rc = letkf_set_schedule(h, bg, bx))) return rc;
  if (cache_path) {
    std::ofstream o(cache_path, std::ios::app);
    o << key.str() << " | graph " << bg << " order " << bx << " ms_per_frame " << best / frames << "\n";
  }
  return LETKF_OK;
}

int letkf_eigh_spd(const double *A_dev, int32_t m, int32_t batch, double tol, int32_t max_sweeps,
                   double *Q_dev, double *lam_dev, int32_t *sweeps_dev, void *stream) {
  if (!A_dev || !Q_dev || !lam_dev || m < 1 || m > 64 || batch < 0)
    return fail(LETKF_E_INVAL, "bad argument");
  if (batch == 0) return LETKF_OK;
  HIPCHK(letkf_launch_eigh(A_dev, m, batch, tol > 0 ? tol : 1e-12, max_sweeps > 0 ? max_sweeps : 30,
                           Q_dev, lam_dev, sweeps_dev, (hipStream_t)stream));
  return LETKF_OK;
}


// ------------------------------------------------------------------ adjoint
extern "C++" {
static int ensure_adjoint(letkf_handle *h) {
  if (!h->adj_ok)
    return fail(LETKF_E_INVAL, "the adjoint needs " + std::to_string(h->adj_lds) +
                                   " bytes of LDS per workgroup, more than the device allows");
  if (h->d_theta) return LETKF_OK;
  const size_t T = h->esize;
  const size_t items = std::max<size_t>(h->items.size(), 1);
  if (hipMalloc(&h->d_xpbar, std::max<size_t>((size_t)h->total_x * T, 16)) != hipSuccess ||
      hipMalloc((void **)&h->d_xbbar, std::max<size_t>((size_t)h->total_nodes * 8, 16)) != hipSuccess ||
      hipMalloc(&h->d_ybar, std::max<size_t>((size_t)h->total_obs * kLanes * T, 16)) != hipSuccess ||
      hipMalloc((void **)&h->d_dbar, std::max<size_t>((size_t)h->total_obs * 8, 16)) != hipSuccess ||
      hipMalloc((void **)&h->d_theta, items * 4 * 8) != hipSuccess)
    return fail(LETKF_E_NOMEM, "hipMalloc of the adjoint buffers failed");
  return LETKF_OK;
}
}  // extern "C++"

int letkf_residual_variance(letkf_handle *h, const void *xa_dev, const void *truth_dev,
                            const double *weights_dev, double *acc_dev, void *stream) {
  if (!h || !truth_dev || !acc_dev) return fail(LETKF_E_INVAL, "NULL argument");
  hipSetDevice(h->device);
  const void *x = xa_dev ? xa_dev : h->d_xa[h->cur];
  HIPCHK(letkf_launch_resvar(h->fp64, h->d_desc, h->n_inst, x, truth_dev,
                             weights_dev ? weights_dev : h->d_ones, h->d_stats, acc_dev,
                             (hipStream_t)stream));
  return LETKF_OK;
}

int letkf_residual_variance_adjoint(letkf_handle *h, const void *xa_dev, const void *truth_dev,
                                    const double *weights_dev, void *xbar_dev, void *stream) {
  if (!h || !truth_dev || !xbar_dev) return fail(LETKF_E_INVAL, "NULL argument");
  hipSetDevice(h->device);
  hipStream_t s = (hipStream_t)stream;
  const void *x = xa_dev ? xa_dev : h->d_xa[h->cur];
  const double *w = weights_dev ? weights_dev : h->d_ones;
  HIPCHK(letkf_launch_resvar(h->fp64, h->d_desc, h->n_inst, x, truth_dev, w, h->d_stats, nullptr, s));
  HIPCHK(letkf_launch_resvar_adjoint(h->fp64, h->d_desc, h->n_inst, x, truth_dev, w, h->d_stats,
                                     xbar_dev, h->max_nodes, s));
  return LETKF_OK;
}

extern "C++" {
template <typename T>
static AdjArgsHost<T> make_adj_args(letkf_handle *h, const void *xa_prev, const void *V,
                                    uint32_t frame, const void *y, void *xbar) {
  AdjArgsHost<T> D;
  std::memset(&D, 0, sizeof(D));
  D.F = make_args<T>(h, true, V, y, 0, 0);
  D.F.x_in = (const T *)xa_prev;
  D.F.x_out = nullptr;
  D.F.x_mean = nullptr;
  D.F.xcd_order = 0;
  D.F.order = nullptr;
  // the adjoint goes through the eigenvectors themselves: converge them further
  // than the forward's transform needs
  D.F.jtol = h->fp64 ? h->jtol : std::min(h->jtol, 1e-6);
  D.F.frame = nullptr;
  set_offsets(D.F, h->off);
  D.xbar = (const T *)xbar;
  D.xpbar = (T *)h->d_xpbar;
  D.xbbar = h->d_xbbar;
  D.ybar = (T *)h->d_ybar;
  D.dbar = h->d_dbar;
  D.theta = h->d_theta;
  D.frame = frame;
  D.off_q = h->adj_off[0];
  D.off_sa = h->adj_off[1];
  return D;
}
}  // extern "C++"

int letkf_adjoint(letkf_handle *h, const void *xa_prev_dev, const void *V_dev, uint32_t frame,
                  const void *y_dev, void *xbar_dev, double *theta_bar_dev, void *stream) {
  if (!h || !xa_prev_dev || !y_dev || !xbar_dev || !theta_bar_dev)
    return fail(LETKF_E_INVAL, "NULL argument");
  if (h->any_loop) return fail(LETKF_E_INVAL, "no adjoint for the closed-loop model");
  if (h->any_ar2) return fail(LETKF_E_INVAL, "no adjoint for the AR(2) model");
  if (h->any_blend) return fail(LETKF_E_INVAL, "no adjoint for the blend-mode gather");
  if (h->transform == kAnalysisCl) return fail(LETKF_E_INVAL, "no adjoint for covariance localisation");
  if (h->any_refit) return fail(LETKF_E_INVAL, "no adjoint with the online refit");
  if (h->wide) return fail(LETKF_E_INVAL, "no adjoint for the wide analysis (m > 64 or a patch over 64 nodes)");
  int rc = check_noise(h, V_dev);
  if (rc) return rc;
  hipSetDevice(h->device);
  if ((rc = ensure_adjoint(h))) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int grid = (int)h->items.size();
  // the piston removal came last in the frame: its adjoint first
  if ((rc = launch_piston_seq(h, {3, 1, 4}, nullptr, xbar_dev, s))) return rc;
  if (h->fp64) {
    auto D = make_adj_args<double>(h, xa_prev_dev, V_dev, frame, y_dev, xbar_dev);
    if (sizeof(D) != letkf_adjoint_args_size(1)) return fail(LETKF_E_DEVICE, "argument layout mismatch");
    HIPCHK(letkf_launch_adjoint(1, &D, grid, h->adj_lds, s));
  } else {
    auto D = make_adj_args<float>(h, xa_prev_dev, V_dev, frame, y_dev, xbar_dev);
    if (sizeof(D) != letkf_adjoint_args_size(0)) return fail(LETKF_E_DEVICE, "argument layout mismatch");
    HIPCHK(letkf_launch_adjoint(0, &D, grid, h->adj_lds, s));
  }
  HIPCHK(letkf_launch_adjoint_nodes(h->fp64, h->d_desc, h->n_inst, h->d_node_adj, h->d_slot_off,
                                    h->d_slots, h->d_xpbar, h->d_xbbar, h->d_ybar, h->d_dbar,
                                    xbar_dev, h->max_nodes, s));
  HIPCHK(letkf_launch_theta_sum(h->d_dom_base, h->n_inst, h->d_theta, theta_bar_dev, s));
  return LETKF_OK;
}


// The adjoint's per-call buffers carved from the fixed device scratch, 256-byte
// aligned: X' adjoint, x_b adjoint, slope slots, innovation slots, per-item
// partials.  Returns the bytes needed.
extern "C++" {
static size_t noalloc_layout(const letkf_handle *h, unsigned char *base, void **xp, double **xb, void **yb,
                             double **db, double **th) {
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t T = h->esize, items = std::max<size_t>(h->items.size(), 1);
  size_t o = 0;
  const size_t o_xp = o; o += up(std::max<size_t>((size_t)h->total_x * T, 16));
  const size_t o_xb = o; o += up(std::max<size_t>((size_t)h->total_nodes * 8, 16));
  const size_t o_yb = o; o += up(std::max<size_t>((size_t)h->total_obs * kLanes * T, 16));
  const size_t o_db = o; o += up(std::max<size_t>((size_t)h->total_obs * 8, 16));
  const size_t o_th = o; o += up(items * 4 * 8);
  if (base) {
    *xp = base + o_xp;
    *xb = (double *)(base + o_xb);
    *yb = base + o_yb;
    *db = (double *)(base + o_db);
    *th = (double *)(base + o_th);
  }
  return o;
}
}  // extern "C++"

int letkf_adjoint_noalloc(letkf_handle *h, const void *xa_prev_dev, const void *V_dev, uint32_t frame,
                          const void *y_dev, void *xbar_dev, double *theta_bar_dev, void *stream) {
  if (!h || !xa_prev_dev || !y_dev || !xbar_dev || !theta_bar_dev)
    return fail(LETKF_E_INVAL, "NULL argument");
  if (h->any_loop) return fail(LETKF_E_INVAL, "no adjoint for the closed-loop model");
  if (h->any_ar2) return fail(LETKF_E_INVAL, "no adjoint for the AR(2) model");
  if (h->any_blend) return fail(LETKF_E_INVAL, "no adjoint for the blend-mode gather");
  if (h->transform == kAnalysisCl) return fail(LETKF_E_INVAL, "no adjoint for covariance localisation");
  if (h->any_refit) return fail(LETKF_E_INVAL, "no adjoint with the online refit");
  if (h->wide) return fail(LETKF_E_INVAL, "no adjoint for the wide analysis (m > 64 or a patch over 64 nodes)");
  if (!h->adj_ok)
    return fail(LETKF_E_INVAL, "the adjoint needs more LDS per workgroup than the device allows");
  int rc = check_noise(h, V_dev);
  if (rc) return rc;
  const size_t need = noalloc_layout(h, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
  if (need > letkf_noalloc_scratch_bytes())
    return fail(LETKF_E_INVAL, "letkf_adjoint_noalloc: the handle needs " + std::to_string(need) +
                                   " bytes of adjoint scratch, more than the fixed " +
                                   std::to_string(letkf_noalloc_scratch_bytes()) + " (use letkf_adjoint)");
  HIPCHK(hipSetDevice(h->device));
  void *base = nullptr;
  HIPCHK(letkf_noalloc_scratch(h->device, &base));
  void *xp = nullptr, *yb = nullptr;
  double *xb = nullptr, *db = nullptr, *th = nullptr;
  noalloc_layout(h, (unsigned char *)base, &xp, &xb, &yb, &db, &th);
  hipStream_t s = (hipStream_t)stream;
  const int grid = (int)h->items.size();
  // the piston step's adjoint first (its per-item buffers belong to the
  // handle, allocated at create); argument blocks on the stack
  if (h->any_piston) {
    for (int which : {3, 1, 4}) {
      int gx, gy;
      letkf_piston_grid(which, (int)h->items.size(), h->n_inst, h->max_nodes, h->max_elems, &gx, &gy);
      if (h->fp64) {
        auto P = make_piston_args<double>(h, nullptr, xbar_dev);
        if (sizeof(P) != letkf_piston_args_size(1)) return fail(LETKF_E_DEVICE, "piston argument layout mismatch");
        HIPCHK(letkf_launch_piston(1, which, &P, gx, gy, s));
      } else {
        auto P = make_piston_args<float>(h, nullptr, xbar_dev);
        if (sizeof(P) != letkf_piston_args_size(0)) return fail(LETKF_E_DEVICE, "piston argument layout mismatch");
        HIPCHK(letkf_launch_piston(0, which, &P, gx, gy, s));
      }
    }
  }
  if (h->fp64) {
    auto D = make_adj_args<double>(h, xa_prev_dev, V_dev, frame, y_dev, xbar_dev);
    D.xpbar = (double *)xp;
    D.xbbar = xb;
    D.ybar = (double *)yb;
    D.dbar = db;
    D.theta = th;
    if (sizeof(D) != letkf_adjoint_args_size(1)) return fail(LETKF_E_DEVICE, "argument layout mismatch");
    HIPCHK(letkf_launch_adjoint(1, &D, grid, h->adj_lds, s));
  } else {
    auto D = make_adj_args<float>(h, xa_prev_dev, V_dev, frame, y_dev, xbar_dev);
    D.xpbar = (float *)xp;
    D.xbbar = xb;
    D.ybar = (float *)yb;
    D.dbar = db;
    D.theta = th;
    if (sizeof(D) != letkf_adjoint_args_size(0)) return fail(LETKF_E_DEVICE, "argument layout mismatch");
    HIPCHK(letkf_launch_adjoint(0, &D, grid, h->adj_lds, s));
  }
  HIPCHK(letkf_launch_adjoint_nodes(h->fp64, h->d_desc, h->n_inst, h->d_node_adj, h->d_slot_off, h->d_slots,
                                    xp, xb, yb, db, xbar_dev, h->max_nodes, s));
  HIPCHK(letkf_launch_theta_sum(h->d_dom_base, h->n_inst, th, theta_bar_dev, s));
  return LETKF_OK;
}

int letkf_set_timing(letkf_handle *h, int32_t enable) {
  if (!h) return fail(LETKF_E_INVAL, "NULL handle");
  h->timing = enable != 0;
  h->tev_used = 0;
  return LETKF_OK;
}

int letkf_analysis_times(letkf_handle *h, float *ms, int32_t max, int32_t *count) {
  if (!h || !count || (max > 0 && !ms)) return fail(LETKF_E_INVAL, "NULL argument");
  hipSetDevice(h->device);
  const int n = (int)std::min<size_t>(h->tev_used, (size_t)std::max(max, 0));
  for (int i = 0; i < n; ++i) {
    HIPCHK(hipEventSynchronize(h->tev[i].second));
    HIPCHK(hipEventElapsedTime(&ms[i], h->tev[i].first, h->tev[i].second));
  }
  *count = (int32_t)h->tev_used;
  h->tev_used = 0;
  return LETKF_OK;
}

}  // extern "C"
