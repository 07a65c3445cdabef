// Device-side descriptors shared by the host planner and the gfx950 kernels.
#pragma once
#include <stdint.h>

namespace letkf {

constexpr int kLanes = 64;        // one wavefront per local analysis
constexpr int kMaxObsSub = 64;    // (b + 2h)^2 observation subapertures at most
constexpr int kMaxOwned = 64;     // (b + 1)^2 owned nodes at most
constexpr int kMaxPatch = 64;     // owned nodes + every corner of the region
constexpr int kYsStride = 80;     // row stride of K-major MFMA operands (no bank conflicts)
constexpr int kXsStride = 65;     // row stride of node rows (lane = row reads)
constexpr int kAnalysisCl = 8;    // analysis-kernel selector of covariance localisation (after the transforms)
constexpr int kAnalysisWide = 16;  // selector of the wide-shape analysis: kAnalysisWide + its 16-column blocks
constexpr int kMaxPatchWide = 128;  // node patch of the wide analysis ((b + 2h + 1)^2 <= 121)
constexpr int kMaxObsSubWide = 100; // its observation subapertures ((b + 2h)^2 <= 100)
constexpr int kMaxMembers = 128;    // ensemble size of the wide analysis
constexpr int kClXtStride = 66;   // covariance localisation: row stride of the FP64 transposed patch

// One adaptive-optics instance.
struct InstDesc {
  int64_t x_off;       // element offset of [node][m] ensemble
  int64_t y_off;       // offset of its slopes (and of its r_diag entries)
  int64_t node_off;    // offset of its node_ij / node tables
  int64_t bank_off;    // element offset of its noise bank (-1: none)
  int32_t n_nodes, n_slopes, n_subaps, m;
  int32_t bank_screens, bank_side;
  uint32_t seed_lo, seed_hi;
  uint32_t instance;
  int32_t piston;      // 1: differential-piston removal after the gather
  int32_t model;       // 0: delay-free phase state; 1: closed loop (delayed slopes, DM terms)
  int32_t blend;       // 1: blend-mode gather (every patch row staged, aligned and blended)
  double a, rho, r_scale, taper_c;
  double a2;           // AR(2): X_b = a X_a(k) + a2 X_a(k-1) + V (0: AR(1))
  double vscale;       // factor on the model noise V (1; the online refit sets it)
};

// Online AR(1) refit of one instance: the forgetting least-squares sums of the
// lag-1 pairs of analysis means (piston removed) and the model it feeds.
struct RefitState {
  double s01, s11;     // sum f^j <x_k - <x_k>, x_{k-1} - <x_{k-1}>>, sum f^j |x_{k-1} - <x_{k-1}>|^2
  double f;            // forgetting factor in (0, 1]; 0: the instance does not refit
  double a0;           // the configured coefficient (the model noise was drawn for it)
  double a_max;        // upper clip of the fitted coefficient
  int64_t frames;      // frames folded in
};

// One term of a domain's piston right-hand side: a subaperture two or more
// domains share, with the summed stencil coefficients (x and y slope) of the
// domain's own corners.
struct PistonTerm {
  int32_t c[4];        // global node index of corners a, b, c, d
  int32_t yx, yy;      // global slope index of its x and y slope
  float cx, cy;        // coefficients (multiples of 1/2)
};

// What the piston step of one work item reads, in one record: its row of
// M^+, where its owned rows are, and its instance's domains.
struct PistonItem {
  int64_t row;         // offset of the item's row of M^+ in the M^+ array
  int64_t x_off;       // the instance's offset into the ensemble
  int32_t b0, nd;      // the instance's first item and number of domains
  int32_t patch_off, n_own;
  int32_t m, piston;   // ensemble size; 0: no piston removal for the instance
};

// One (instance, domain) work item.  Patch entries 0..n_own-1 are the owned
// nodes in ascending order; the rest are the other corners of the region.
struct DomItem {
  int32_t inst;
  int32_t dom;         // domain number within the instance
  int32_t n_own, n_patch, n_obs;   // n_obs observation subapertures (p_l = 2 n_obs)
  int32_t patch_off;   // into patch_node
  int32_t obs_off;     // into obs_corner / obs_sub / obs_dist
  int32_t pad0;
};

}  // namespace letkf
