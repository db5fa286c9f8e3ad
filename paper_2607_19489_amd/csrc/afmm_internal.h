// Internal declarations shared by the host plan builder and the HIP kernels.
//
// Units.  Every level works in its own cell units so that FP32 coefficients
// stay O(1) at any depth:
//   S~_f[r]_a = sum_{leaves x under r} m_x ((x_x - c_r) / h_f)^a        (multipoles)
//   L~_f[r]_b = h_f^(1+|b|) d^b(phi/G) at c_r                          (local expansions)
//   phi_c = (G / h_l) phi~_c,   a_c = (G / h_l^2) a~_c                   (outputs)
// With these, every translation operator is a fixed table on unit offsets:
//   M2M  S~_a[r] = sum_o sum_{k<=a} C(a,k) d_o^(a-k) 2^-|k| S~_k[child o],  d_o = (o - 1/2)/2
//   M2L  L~_b[y] = sum_a (-1)^|a|/a! 2^|a| D~_{a+b}(R~) S~_a[s],  R~ = -2(s - F) + o_y - 1/2
//   L2L  L~_b[y] = 2^(-1-|b|) sum_g u^g/g! L~_{b+g}[F],  u = (o_y - 1/2)/2
//   M2P  phi~ = sum_a (-1)^|a|/a! 2^|a| D~_a(R~) S~_a,  a~_i = -sum_{|a|<p} (...) D~_{a+e_i} S~_a
//   L2P  phi~ = 1/2 sum_b L~_b u^b/b!,  a~_i = -1/4 sum_{b_i>0} L~_b u^(b-e_i)/(b-e_i)!
// where D~_g = d^g(-1/r) on unit offsets (Sec. 2 Eqs. eq:M2M_general, eq:M2L, eq:L2L).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <exception>
#include <memory>
#include <thread>
#include <vector>

#include "afmm.h"
#include "host_pool.h"

namespace afmm {

// Morton key of cell (x, y, z): bit b of x, y, z at bits 3b, 3b + 1, 3b + 2;
// every level of a plan is ordered by it.
inline uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  auto spread = [](uint64_t v) {
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
  };
  return spread(x) | (spread(y) << 1) | (spread(z) << 2);
}

constexpr int kMaxLevel = 21;
constexpr int kPMax = 8;
constexpr int kKMax = 165;          // C(kPMax + 3, 3)
constexpr int kNumD = 343;          // offsets d in [-3, 3]^3

__host__ __device__ constexpr int nmi(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }
// number of pairs (a, k) with k <= a componentwise and |a| <= p: C(p + 6, 6)
__host__ __device__ constexpr int nmi_entries(int p) {
  return (p + 1) * (p + 2) * (p + 3) * (p + 4) * (p + 5) * (p + 6) / 720;
}

// Position of multi-index (a, b, c) in the degree-graded order (degree, then a
// descending, then b descending).
__host__ __device__ constexpr int mi_index(int a, int b, int c) {
  return (a + b + c) * (a + b + c + 1) * (a + b + c + 2) / 6 + (b + c) * (b + c + 1) / 2 + c;
}

// Layout of the scaled source copies (S32 / Sc64).  The MFMA kernels read the
// B operand straight into registers: lane group g (lane >> 4) of a 16x16x4
// step kb holds coefficient k = 4 kb + g.  A lane group needs STP steps
// (STP = ceil(K/4) rounded up to whole 16-byte vectors of VW = 16/bytes
// values); its vector j holds steps VW j .. VW j + VW - 1.  The row stores the
// vectors j-major: vector j of lane group g at (4 j + g) VW, so one 16-byte
// load per lane (vector j for all 4 lane groups of a source) reads 64
// contiguous bytes of each source row.  Coefficient k therefore sits at
// ((k >> 2) / VW) 4 VW + (k & 3) VW + (k >> 2) % VW; unused slots are 0.
__host__ __device__ constexpr int src_stp(int p, int bytes) {
  return (((nmi(p) + 3) / 4) + (16 / bytes) - 1) / (16 / bytes) * (16 / bytes);
}
__host__ __device__ constexpr int src_row(int p, int bytes) { return 4 * src_stp(p, bytes); }
__host__ __device__ constexpr int src_pos(int k, int bytes) {
  return ((k >> 2) / (16 / bytes)) * 4 * (16 / bytes) + (k & 3) * (16 / bytes) + (k >> 2) % (16 / bytes);
}
// element offset of vector j of lane group g in a source row
__host__ __device__ constexpr int src_vec(int j, int g, int bytes) { return (4 * j + g) * (16 / bytes); }

// D~ rows of one source offset in the layout the MFMA kernels stage in LDS:
// row o (child octant) at o * dstage_ks(p), coefficients g < K then zeros up
// to the stride, one zero slot at 8 * dstage_ks(p), zero padding to whole
// 16-byte vectors for every lane of a wave.  Copied to LDS as is.  The row
// stride is chosen per order (at least K rounded up to 4, same padded length)
// to spread the A-operand gathers of M2P and M2L (8 rows x derivative-shifted
// coefficient indices per lane) over the LDS banks; chosen by counting bank
// conflicts of those offset tables for 32- and 64-bank LDS models.
__host__ __device__ constexpr int dstage_ks(int p) {
  return p == 1 ? 6 : p == 2 ? 30 : p == 3 ? 28 : p == 4 ? 52 : p == 5 ? 57 : p == 6 ? 93 : p == 7 ? 121 : 185;
}
__host__ __device__ constexpr int dstage_len(int p, int bytes) {
  return (8 * dstage_ks(p) + 1 + 64 * (16 / bytes) - 1) / (64 * (16 / bytes)) * (64 * (16 / bytes));
}

// Near field of one group as a fixed linear map (Sec. 3.2, Alg. 4): the 8
// targets (rows c * 8 + o, c = phi, ax, ay, az) take P2P from the 216 children
// of the father's 27 neighbours (columns 8 e + o'), P2P from the 27
// neighbours themselves when they are leaves one level coarser (columns
// 216 + e), and L2P from the father's local expansion (columns 243 + b).
// Columns are padded to whole 16-byte vectors of MFMA steps for both
// precisions; the operator is stored per lane of the 16x16x4 A operand:
// element [t][kb / VW][lane][kb % VW] is row 16 t + (lane & 15), column
// 4 kb + (lane >> 4), VW = 16 / bytes.
constexpr int kNearLeafCols = 216;
constexpr int kNearCoarseCols = 27;
__host__ __device__ constexpr int near_cols(int p) { return (kNearLeafCols + kNearCoarseCols + nmi(p) + 15) / 16 * 16; }
__host__ __device__ constexpr int near_ksteps(int p) { return near_cols(p) / 4; }

// Interaction-list taps per octant class: the children of the father's 27
// neighbours (216) less the cell's own 27 neighbours.
constexpr int kTapsPerClass = 189;

// Work items of one launch split into 8 contiguous ranges, one per XCD (the
// hardware deals workgroups to the XCDs round-robin): workgroup b runs item
// start[b % 8] + b / 8 if that is below start[b % 8 + 1].  Ranges of equal
// estimated work rather than equal length keep every XCD busy when the work
// per item varies; each XCD still reads a contiguous run of tiles.
struct XcdRanges {
  int32_t start[9] = {};
  int32_t grid() const {
    int32_t m = 0;
    for (int x = 0; x < 8; ++x) m = start[x + 1] - start[x] > m ? start[x + 1] - start[x] : m;
    return 8 * m;
  }
};

// Per-level device view.  Level l holds the children of the refined cells of
// level l - 1 in Morton order, so cell index c has father refined rank c >> 3
// and octant c & 7 (o = ox + 2 oy + 4 oz), and refined rank r owns children
// 8r .. 8r+7.  Neighbour index e = (ex+1) + 3(ey+1) + 9(ez+1).
struct LevelDev {
  int32_t n = 0;             // cells
  int32_t nref = 0;          // refined cells
  const int32_t* rank = nullptr;     // [n] refined rank or -1 (leaf)
  const int32_t* slot = nullptr;     // [n] caller slot (flat index) or -1 (cells above levelmin)
  const int32_t* refcell = nullptr;  // [nref] cell index of refined rank r
  const int32_t* nbr = nullptr;      // [nref][27] neighbour cell index at this level, -1 outside box
  double* mass = nullptr;            // [n] leaf masses of this solve (0 for refined cells)
  double* S64 = nullptr;             // [nref][K] multipoles (FP64), used by the upward pass
  float* S32 = nullptr;              // [nref][src_row(p, 4)] source copy (-1)^|a|/a! 2^|a| S~_a, FP32
                                     // (mixed form), in the lane-group layout above
  double* Sc64 = nullptr;            // [nref][src_row(p, 8)] same source copy in FP64
  double* L64 = nullptr;             // [nref][K] local expansions (FP64 levels)
  float* L32 = nullptr;              // [nref][K] local expansions (FP32 levels)
  void* part = nullptr;              // [npart][nref][32] intermediate-field partials of the leaf children (T of the
                                     // leaf level), one set per M2P tap range
  int32_t npart = 0;
  size_t part_bytes = 0, Lpart_bytes = 0;
  void* Lpart = nullptr;             // [nsplit][nref][K] M2L tap-range partial sums (T of the level), if split
  // adjoint pass (FP64, allocated by the first adjoint call)
  double* tbar = nullptr;            // [n][4] unit-form bars of the target leaves (phi, ax, ay, az)
  double* mbar = nullptr;            // [n] mass bars of the leaves
  double* sbar = nullptr;            // [nref][K] source-copy bar, then multipole bar
  double* lbar = nullptr;            // [nref][K] local-expansion bar
  void* tbT = nullptr;               // [nref][32] target bars of the leaf children, B of the transposed M2P (T)
  void* lbarT = nullptr;             // [nref][src_row] local-expansion bar, B of the transposed M2L (T, lane-group layout)
};

template <typename T>
struct TablesDev {
  const T* Dstage = nullptr;  // [kNumD][dstage_len(p, sizeof(T))] D~ at R~ = -2d + o - 1/2, 8 rows per d,
                              // in the LDS stage layout of the MFMA kernels
  const T* Dsame = nullptr;   // [kNumD][K]      D~ at integer R~ in [-3,3]^3
  const T* cfac2 = nullptr;   // [K] (-1)^|a|/a! 2^|a|
  const T* cfacn = nullptr;   // [K] 2^-|a|: same-level M2P from the source copies
  const T* l2lw = nullptr;    // [8][p+1][K] L2L weights 2^(-1-|b|) u^g/g! per child octant and |b|
  const T* l2p = nullptr;     // [8][4][K] L2P weights (phi, ax, ay, az) per child octant
  const T* nearA = nullptr;   // [2][near_ksteps / VW][64][VW] near-field operator, MFMA A layout
  const T* adjNearA = nullptr;  // [216][64] transposed same-level near field (adjoint), MFMA A layout
};

struct CommonDev {
  const int16_t* sumidx = nullptr;  // [K][K] index of a + b (or -1 when |a|+|b| > p)
  const int16_t* up = nullptr;      // [K][3] index of a + e_i (or -1 when |a| = p)
  const int8_t* mi = nullptr;       // [K][4] (a, b, c, |a|)
  const double* binom = nullptr;    // [(kPMax+1)^2] binomial coefficients C(n, k) at n*(kPMax+1)+k
  const double* cfac2 = nullptr;    // [K] (-1)^|a|/a! 2^|a| (FP64), applied to the source copies
  const int32_t* m2m_start = nullptr;  // [K+1] M2M entry range of each coefficient a
  const int32_t* m2m_list = nullptr;   // entries: k | parity(a-k) << 12
  const double* m2m_w = nullptr;       // entry weights C(a,k) 4^-|a-k| 2^-|k|
  const int32_t* m2mT_start = nullptr; // [K+1] the same entries grouped by k (adjoint)
  const int32_t* m2mT_list = nullptr;  // entries: a | parity(a-k) << 12
  const double* m2mT_w = nullptr;
  const int32_t* tapsT = nullptr;      // [8][189] per source octant: e | oF << 5 | d_index << 8 (adjoint)
  const int16_t* adj_m2p_off = nullptr; // [RT * 8][64] A offsets of the transposed M2P
  const int16_t* adj_m2l_off = nullptr; // [steps][64] A offsets (within one D~ row) of the transposed M2L
  const int32_t* l2lT_start = nullptr;  // [K+1] transposed L2L pairs of each coefficient c
  const int32_t* l2lT_list = nullptr;   // b | (c - b) << 8 | |b| << 16 | parity(c - b) << 24
  const double* l2lT_w = nullptr;       // [entries] weight 2^(-1-|b|) u_7^(c-b)/(c-b)! of child 7 (u_7 = +1/4)
};

// Group tiles of the MFMA kernels: NC refined ranks per tile (one parity class,
// -1 padded), tiles of the 8 classes interleaved.
struct MfmaTiles {
  const int32_t* tiles = nullptr;
  int ntiles = 0;
  int nc = 0;
};

struct MfmaTables {
  const int32_t* taps = nullptr;      // [8][189] per parity class: e | o' << 5 | d_index << 8
  const int16_t* m2p_off = nullptr;   // [steps][64] sD offsets of the M2P A operand
  const int16_t* m2l_off = nullptr;   // [steps][64] sD offsets of the M2L A operand
  const int32_t* m2l_tinfo = nullptr; // [NT][2] k-steps and first step of each M2L row tile
};

// Launchers (afmm_kernels.hip).  All return hipGetLastError() of the launch.
// Leaf masses of one level from the caller's slot array; with `snap`, every
// cell's slot value is also copied there (the adaptive-time-step snapshot).
hipError_t launch_gather_mass(const LevelDev& lv, const double* m_src, double* snap, hipStream_t st);
// Drifted masses of a solve with stale trees: out[s] = m[s] + dt * rate[s] for
// the slots [off[i], off[i + 1]) of AMR level i (levels with dt = 0 copied)
struct DriftLevels {
  int n = 0;
  int64_t off[kMaxLevel + 1] = {};
  double dt[kMaxLevel] = {};
};
hipError_t launch_drift(const DriftLevels& d, const double* m, const double* rate, double* out, int64_t nslots,
                        hipStream_t st);
hipError_t launch_copy_slots(const int32_t* slots, int64_t n, const double* src, double* dst,
                             hipStream_t st);
// Batches: forest slot <-> caller arrays.  leafslot/leafhier list every leaf of
// the forest with its hierarchy; base[h] is the hierarchy's first forest slot.
hipError_t launch_batch_in(int64_t nleaf, const int32_t* leafslot, const int32_t* leafhier, const int64_t* base,
                           const double* const* mass, double* m_forest, hipStream_t st);
hipError_t launch_batch_out(int64_t nleaf, const int32_t* leafslot, const int32_t* leafhier, const int64_t* base,
                            const double* phi_forest, const double* acc_forest, double* const* phi,
                            double* const* acc, hipStream_t st);
// Adjoint pass (afmm_adjoint.hip).
hipError_t launch_adj_init(const LevelDev& lv, int target, const double* phib, const double* accb, double sp,
                           double sa, hipStream_t st);
hipError_t launch_adj_zero(double* p, size_t n, hipStream_t st);
// Adjoint near field of level l: the same-level P2P^T of the leaf groups as
// one MFMA product (targets_here only), the coarse and nearest P2P^T of the
// groups in vgrp (those with a leaf neighbour one level coarser or a refined
// near candidate), the near M2P^T of refgrp.
hipError_t launch_adj_near(int p, const int32_t* leafgrp, int nleafgrp, const int32_t* vgrp, int nvgrp,
                           const int32_t* refgrp, int nrefgrp, const LevelDev& lv1, const LevelDev& lv0,
                           const LevelDev& lvp, int targets_here, const TablesDev<double>& t64, const CommonDev& cm,
                           hipStream_t st);
hipError_t launch_adj_l2p(int p, const int32_t* grp, int ngrp, const LevelDev& lv1, const LevelDev& lv0,
                          const TablesDev<double>& t64, const CommonDev& cm, hipStream_t st);
// MFMA forms: tiles of 16 source cells (records: target level, 16 cells); with
// nsplit > 1 the 189 taps of a tile are split over blocks writing partial sets
// into `part` ([nsplit][ntiles * 16][K] FP64), summed in order afterwards.
// Periodic boxes: the level-2 far operator table ([8][kNumD][K] in level-2
// units, cached per order) and its kernel (writes L of the 64 level-2 cells).
std::shared_ptr<const std::vector<double>> periodic_far_table(int p);
hipError_t launch_periodic_far(int p, const LevelDev& lv2, const double* T, const double* cf, const CommonDev& cm,
                               hipStream_t st);
// its transpose: level-2 multipole bars from the level-2 local-expansion bars
hipError_t launch_adj_periodic_far(int p, const LevelDev& lv2, const double* T, const double* cf,
                                   const CommonDev& cm, hipStream_t st);
hipError_t launch_adj_m2p_mfma(int p, bool fp32, const int32_t* tiles, int ntiles, int nsplit, const XcdRanges& xr,
                               const uint8_t* live, double* part,
                               const int32_t* tapsT, const int16_t* aoff, const LevelDev& lvp, const LevelDev& lvs,
                               const LevelDev& lvt, const TablesDev<float>& t32, const TablesDev<double>& t64,
                               hipStream_t st);
hipError_t launch_adj_m2l_mfma(int p, bool fp32, const int32_t* tiles, int ntiles, int nsplit, const XcdRanges& xr,
                               const uint8_t* live, double* part,
                               const int32_t* tapsT, const int16_t* aoff, const LevelDev& lvp, const LevelDev& lvs,
                               const LevelDev& lvt, const TablesDev<float>& t32, const TablesDev<double>& t64,
                               hipStream_t st);
hipError_t launch_adj_l2l(int p, const int32_t* grp, int ngrp, const LevelDev& lv1, const LevelDev& lv0,
                          const TablesDev<double>& t64, const CommonDev& cm, hipStream_t st);
hipError_t launch_adj_down(int p, const int32_t* grp, int ngrp, const LevelDev& lv1, const LevelDev& lv0,
                           int has_parent, const CommonDev& cm, hipStream_t st);
// Mass bars to the caller's slots; cself (the self-potential constant, 0 when
// off) adds the transpose of the self term -cself m of the unit-form potential.
hipError_t launch_adj_out(int p, const LevelDev& lv1, const LevelDev& lv0, int has_parent, int rebuilt,
                          double cself, const CommonDev& cm, double* mbar_out, hipStream_t st);
// Upward pass of FMM level f: the refined cells whose children are all leaves
// (list leaf, P2M only) and the others (list mix, M2M of refined children).
hipError_t launch_upward(int p, const int32_t* leaf, int nleaf, const int32_t* mix, int nmix, const LevelDev& lv,
                         const LevelDev& lvc, const CommonDev& cm, hipStream_t st);
int m2p_columns(int p, bool fp32);
bool m2p_shape_ok(int p, bool fp32, int shape);
int m2p_shape_columns(int shape);
// MFMA launches over a contiguous range [t0, t0 + n) of tile records; each
// record is (target level, NC groups).  lvs is the device array of LevelDev.
hipError_t launch_m2l_taps(int p, bool fp32, const MfmaTiles& mt, int t0, int n, int nsplit, const MfmaTables& tabs,
                           const LevelDev* lvs, const TablesDev<float>& t32, const TablesDev<double>& t64,
                           hipStream_t st);
hipError_t launch_l2l(int p, bool fp32, bool parent_fp32, bool has_parent, int nsplit, const int32_t* grp, int ngrp,
                      const LevelDev& lv1, const LevelDev& lv0, const TablesDev<float>& t32,
                      const TablesDev<double>& t64, const CommonDev& cm, hipStream_t st);
hipError_t launch_m2p(int p, bool fp32, const MfmaTiles& mt, int t0, int n, int nsplit, int shape,
                      const MfmaTables& tabs, const LevelDev* lvs, const TablesDev<float>& t32,
                      const TablesDev<double>& t64, hipStream_t st);
// cself: the self-potential constant (AFMM_SELF_POTENTIAL), 0 when off.
hipError_t launch_near(int p, bool fp32, int l, int l_first, const int32_t* grp, int ngrp, const LevelDev& lv1,
                       const LevelDev& lv0, const LevelDev& lvp, const TablesDev<float>& t32,
                       const TablesDev<double>& t64, const CommonDev& cm, const void* part, const void* nmp,
                       double G, double h, double cself, double* phi, double* acc, hipStream_t st);
// Near-field M2P from the refined level-l cells among the near candidates of
// the groups `grp` (those that have any): partial [nref(l-1)][c * 8 + o].
hipError_t launch_near_m2p(int p, bool fp32, const int32_t* grp, int ngrp, const LevelDev& lv1, const LevelDev& lv0,
                           const LevelDev& lvp, const TablesDev<float>& t32, const TablesDev<double>& t64, void* nmp,
                           hipStream_t st);

}  // namespace afmm
