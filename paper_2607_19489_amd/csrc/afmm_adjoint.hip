// Adjoint (transposed) pass of the adaptive FMM.  The translation products
// (M2P^T, M2L^T) run on MFMA in the precision of the forward kernel of the same
// level; bars are accumulated in FP64.
//
// A solve is a linear map m -> (phi, a).  These kernels apply its transpose:
// given bars (phi_bar, a_bar) on the target leaves they return m_bar, running
// the forward steps backwards with each operator transposed:
//
//   forward                                    adjoint (this file)
//   output scale phi = G/h phi~, a = G/h^2 a~  T_c = (G/h phi_bar, G/h^2 a_bar)  k_adj_init
//   near P2P / nearest P2P (Sec. 3.2)          P2P^T gathered per source leaf     k_adj_near_leaf
//   near M2P from refined level-l cells        M2P^T into the level-l source bar  k_adj_near_m2p
//   L2P (far field)                            L2P^T into the father's L bar      k_adj_l2p
//   M2P, intermediate field                    M2P^T per source cell (MFMA)       k_adj_m2p_mfma
//   L2L (Eq. eq:L2L), top-down                 L2L^T, bottom-up                   k_adj_l2l
//   M2L (Eq. eq:M2L), 189-cell list            M2L^T per source cell (MFMA)       k_adj_m2l_mfma
//   source copy c_a 2^|a| S~_a                 scale of the source bar            k_adj_down
//   M2M (Eq. eq:M2M_general), bottom-up        M2M^T, top-down                    k_adj_down, k_adj_leafup
//   mass gather (slot -> cell)                 scatter (cell -> slot)             k_adj_out
//
// Every relation is gathered from the receiving side, so no atomics are needed
// and the sums run in a fixed order.  The interaction list relation is
// symmetric at one level (s is in F's list iff |parent(s) - parent(F)| <= 1
// and |s - F| >= 2), so a source cell s finds every group F that reads it
// through its own parent's 27 neighbours: 189 "transposed taps" per octant of s.
#include <hip/hip_runtime.h>

#include "afmm_internal.h"
#include "afmm_mfma.h"

namespace afmm {

namespace {

constexpr int kTapsT = 189;

__device__ inline int ax_e(int e, int d) { return (d == 0 ? e % 3 : (d == 1 ? (e / 3) % 3 : e / 9)) - 1; }
__device__ inline int ax_o(int o, int d) { return (o >> d) & 1; }
__device__ inline int dsame_index(int dx, int dy, int dz) { return (dx + 3) + 7 * (dy + 3) + 49 * (dz + 3); }

// Transpose of p2p(): the pair phi~ -= m/|r|, a~ -= m r/|r|^3 (r = target -
// source, target-level units) gives m_bar -= Tphi/|r| + TA.r/|r|^3.
__device__ inline double p2p_adj(double rx, double ry, double rz, const double* __restrict__ tb) {
  const double r2 = rx * rx + ry * ry + rz * rz;
  const double inv = 1.0 / sqrt(r2);
  return -(tb[0] * inv + (tb[1] * rx + tb[2] * ry + tb[3] * rz) * inv * inv * inv);
}

// sign of child octant o in the signed child sum of parity class q
__device__ inline double parity_sign(int q, int o) { return (__popc(q & ~o) & 1) ? -1.0 : 1.0; }


}  // namespace

// Bars of the targets in unit form and zeroed mass bars, one level.
__global__ void k_adj_init(int n, const int32_t* __restrict__ rank, const int32_t* __restrict__ slot, int target,
                           const double* __restrict__ phib, const double* __restrict__ accb, double sp, double sa,
                           double* __restrict__ tbar, double* __restrict__ mbar) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int s = slot[i];
  const bool t = target && rank[i] < 0 && s >= 0;
  tbar[4 * (size_t)i + 0] = t ? sp * phib[s] : 0.0;
  tbar[4 * (size_t)i + 1] = t ? sa * accb[3 * (size_t)s + 0] : 0.0;
  tbar[4 * (size_t)i + 2] = t ? sa * accb[3 * (size_t)s + 1] : 0.0;
  tbar[4 * (size_t)i + 3] = t ? sa * accb[3 * (size_t)s + 2] : 0.0;
  mbar[i] = 0.0;
}

__global__ void k_adj_zero(size_t n, double* __restrict__ p) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// P2P^T for the leaves s of level l from targets one level finer or coarser
// (block = one group F of level l-1 with a leaf child; s = its child o = t &
// 7).  The 216 candidates (children of F's 27 neighbours, or the neighbour
// itself when it is a leaf) are resolved once into LDS; partial sums are
// reduced by shuffles within a wave and through LDS across waves.  Targets
// that read s through a P2P:
//   level l+1 children of a refined level-l n touching s (s is in their near
//     field as a coarse leaf),
//   level l-1 leaves q touching F (s is in q's nearest field).
// The same-level near field (level l leaves among the children of F's
// neighbours) is k_adj_near_mfma.
__global__ __launch_bounds__(256) void k_adj_near_leaf(const int32_t* __restrict__ grp, LevelDev lv1, LevelDev lv0,
                                                       LevelDev lvp) {
  enum { kNone = 0, kCoarse = 1, kLeaf = 2, kRefined = 3 };
  __shared__ int s_kind[216];
  __shared__ int s_idx[216];
  __shared__ double s_red[4][8];
  const int F = grp ? grp[blockIdx.x] : (int)blockIdx.x;
  const int t = threadIdx.x, o = t & 7, j = t >> 3;
  if (t < 216) {
    const int e = t >> 3, op = t & 7;
    const int q = lv1.nbr[(size_t)F * 27 + e];
    int kind = kNone, idx = -1;
    if (q >= 0) {
      const int rq = lv1.rank[q];
      if (rq < 0) {
        if (op == 0) kind = kCoarse, idx = q;
      } else {
        const int n = 8 * rq + op;
        const int rn = lv0.rank[n];
        if (rn < 0) kind = kLeaf, idx = n;
        else kind = kRefined, idx = rn;
      }
    }
    s_kind[t] = kind;
    s_idx[t] = idx;
  }
  __syncthreads();
  const int s = 8 * F + o;
  double acc = 0.0;
  if (lv0.rank[s] < 0) {
    const int sx = ax_o(o, 0), sy = ax_o(o, 1), sz = ax_o(o, 2);
    for (int k = j; k < 216; k += 32) {
      const int kind = s_kind[k];
      if (kind == kNone) continue;
      const int e = k >> 3, op = k & 7;
      const int ex = ax_e(e, 0), ey = ax_e(e, 1), ez = ax_e(e, 2);
      const int idx = s_idx[k];
      if (kind == kCoarse) {
        // nearest field of the coarse leaf q = F + e: r = e - (o - 1/2)/2 in h_(l-1) units
        acc += p2p_adj(ex - (sx - 0.5) * 0.5, ey - (sy - 0.5) * 0.5, ez - (sz - 0.5) * 0.5, lv1.tbar + 4 * (size_t)idx);
        continue;
      }
      const int tx = sx - 2 * ex - ax_o(op, 0), ty = sy - 2 * ey - ax_o(op, 1), tz = sz - 2 * ez - ax_o(op, 2);
      if (kind == kRefined && max(abs(tx), max(abs(ty), abs(tz))) <= 1) {
        for (int o2 = 0; o2 < 8; ++o2)
          acc += p2p_adj(ax_o(o2, 0) - 0.5 - 2.0 * tx, ax_o(o2, 1) - 0.5 - 2.0 * ty, ax_o(o2, 2) - 0.5 - 2.0 * tz,
                         lvp.tbar + 4 * (size_t)(8 * idx + o2));
      }
    }
  }
#pragma unroll
  for (int w = 8; w <= 32; w <<= 1) acc += __shfl_xor(acc, w, 64);
  if ((t & 63) < 8) s_red[t >> 6][o] = acc;
  __syncthreads();
  if (t < 8 && lv0.rank[s] < 0) lv0.mbar[s] += s_red[0][o] + s_red[1][o] + s_red[2][o] + s_red[3][o];
}

// Same-level near field transposed (the P2P^T of the forward near operator's
// leaf columns): for a source group F (level l-1) its children receive
//   m_bar[8F + op] += sum_{e', o, q} W[op][32 e' + 4 o + q] T[8 F' + o][q],
// F' = F's neighbour e' (a refined cell, else no term), T the unit-form target
// bars, W = adjNearA (the forward weights of slot 8 (26 - e') + op).  As an
// FP64 MFMA product [16 x 864] . [864 x 16 groups] with rows 8..15 zero; the
// 4 waves of a block take a quarter of the 216 steps each and wave 0 adds
// the others' accumulators in order.
__global__ __launch_bounds__(256) void k_adj_near_mfma(const int32_t* __restrict__ grp, int ngrp, LevelDev lv1,
                                                       LevelDev lv0, const double* __restrict__ W) {
  constexpr int NKB = 216, KW = NKB / 4;
  __shared__ int sF[16];
  __shared__ int sRF[16 * 27];
  __shared__ double sAcc[3][4][64];
  const int ntiles = (ngrp + 15) / 16;
  const int tile = xcd_tile(ntiles);
  if (tile >= ntiles) return;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63, n = lane & 15, g = lane >> 4;
  if (t < 16) sF[t] = 16 * tile + t < ngrp ? grp[16 * tile + t] : -1;
  __syncthreads();
  for (int i = t; i < 16 * 27; i += 256) {
    const int c = i / 27, e = i - 27 * c;
    const int F = sF[c];
    int v = -1;
    if (F >= 0) {
      const int q = lv1.nbr[(size_t)F * 27 + e];
      if (q >= 0) v = lv1.rank[q];
    }
    sRF[i] = v;
  }
  __syncthreads();
  gptr<double> tb = as_global(lv0.tbar);
  gptr<double> Wg = as_global(W);
  f64x4 acc = {0, 0, 0, 0};
  double bv[KW];
#pragma unroll
  for (int i = 0; i < KW; ++i) {
    const int k = 4 * (KW * w + i) + g;
    const int rF = sRF[n * 27 + (k >> 5)];
    const double v = tb[32 * (size_t)(rF >= 0 ? rF : 0) + (k & 31)];
    bv[i] = rF >= 0 ? v : 0.0;
  }
#pragma unroll
  for (int i = 0; i < KW; ++i) acc = mfma16(Wg[(size_t)(KW * w + i) * 64 + lane], bv[i], acc);
  if (w > 0)
#pragma unroll
    for (int r = 0; r < 4; ++r) sAcc[w - 1][r][lane] = acc[r];
  __syncthreads();
  const int F = sF[n];
  if (w > 0 || F < 0) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double v = acc[r] + sAcc[0][r][lane] + sAcc[1][r][lane] + sAcc[2][r][lane];
    const int op = acc_row<double>(g, r);
    if (op >= 8) continue;
    const int s = 8 * F + op;
    if (lv0.rank[s] < 0) lv0.mbar[s] += v;
  }
}

// Near-field M2P^T: a refined level-l cell s is read, through 2^-|a| times its
// source copy, by the level-l leaves n among the children of F's neighbours
// that do not touch s.  Source-copy bar of s += cfacn_a (D_a T_phi - sum_i
// D_(a+e_i) T_i) with D = D~ at n - s.
template <int P>
__global__ __launch_bounds__(256) void k_adj_near_m2p(const int32_t* __restrict__ grp, LevelDev lv1, LevelDev lv0,
                                                      const double* __restrict__ Dsame,
                                                      const double* __restrict__ cfacn,
                                                      const int16_t* __restrict__ up) {
  constexpr int K = nmi(P), K1 = nmi(P - 1);
  __shared__ int s_slot[216];     // candidate slots 8 e + op with a leaf, in slot order
  __shared__ double s_tb[216][4]; // their target bars
  __shared__ int s_ref[8];
  __shared__ int s_cnt[4];
  const int F = grp ? grp[blockIdx.x] : (int)blockIdx.x;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  if (t < 8) s_ref[t] = lv0.rank[8 * F + t];
  int v = -1;
  if (t < 216) {
    const int e = t >> 3, op = t & 7;
    const int q = lv1.nbr[(size_t)F * 27 + e];
    if (q >= 0) {
      const int rq = lv1.rank[q];
      if (rq >= 0 && lv0.rank[8 * rq + op] < 0) v = 8 * rq + op;
    }
  }
  // leaf candidates compacted in slot order (ballot per wave, wave counts in LDS)
  const uint64_t m = __ballot(v >= 0);
  if (lane == 0) s_cnt[w] = __popcll(m);
  // no leaf among the candidates (inside a refined region): nothing reads the
  // group's refined children here
  if (!__syncthreads_or(v >= 0)) return;
  int base = 0, nlist = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    base += u < w ? s_cnt[u] : 0;
    nlist += s_cnt[u];
  }
  if (v >= 0) {
    const int pos = base + __popcll(m & ((1ull << lane) - 1ull));
    s_slot[pos] = t;
#pragma unroll
    for (int c = 0; c < 4; ++c) s_tb[pos][c] = lv0.tbar[4 * (size_t)v + c];
  }
  __syncthreads();
  bool any = false;
  for (int o = 0; o < 8; ++o) any |= s_ref[o] >= 0;
  if (!any) return;
  gptr<double> Dg = as_global(Dsame);
  for (int i = t; i < 8 * K; i += 256) {
    const int o = i / K, a = i - o * K;
    const int rs = s_ref[o];
    if (rs < 0) continue;
    const int u0 = a < K1 ? up[3 * a + 0] : 0, u1 = a < K1 ? up[3 * a + 1] : 0, u2 = a < K1 ? up[3 * a + 2] : 0;
    double acc = 0.0;
    for (int j = 0; j < nlist; ++j) {
      const int k = s_slot[j];
      const int e = k >> 3, op = k & 7;
      const int dx = 2 * ax_e(e, 0) + ax_o(op, 0) - ax_o(o, 0);
      const int dy = 2 * ax_e(e, 1) + ax_o(op, 1) - ax_o(o, 1);
      const int dz = 2 * ax_e(e, 2) + ax_o(op, 2) - ax_o(o, 2);
      if (max(abs(dx), max(abs(dy), abs(dz))) <= 1) continue;
      gptr<double> D = Dg + (size_t)dsame_index(dx, dy, dz) * K;
      double v2 = D[a] * s_tb[j][0];
      if (a < K1) v2 -= D[u0] * s_tb[j][1] + D[u1] * s_tb[j][2] + D[u2] * s_tb[j][3];
      acc += v2;
    }
    lv0.sbar[(size_t)rs * K + a] += cfacn[a] * acc;
  }
}

// L2P^T: the far field of the leaf children of F (a group with a leaf child)
// reads L~[F] (level l-1).  The child offsets have components +-1/4, so the
// weight of child o for quantity q (phi, a_x, a_y, a_z) at coefficient b is
// that of child 7 times (-1)^popcount(~o & pi), pi the parity of b (phi) or
// of b - e_i (a_i): the 8 children's target bars are folded per quantity into
// Y_q[pi] = sum_o (-1)^popcount(~o & pi) T_o[q] first.
template <int P>
__global__ __launch_bounds__(256) void k_adj_l2p(const int32_t* __restrict__ grp, int ngrp, LevelDev lv1, LevelDev lv0,
                                                 const double* __restrict__ l2p, const int8_t* __restrict__ mi) {
  constexpr int K = nmi(P);
  constexpr int GB = 256 / K > 0 ? 256 / K : 1;  // groups per block
  __shared__ double s_t[GB][32];
  __shared__ double sY[GB][4][8];
  const int t = threadIdx.x;
  const int g0 = blockIdx.x * GB;
  for (int i = t; i < GB * 32; i += 256) {
    const int gi = g0 + (i >> 5);
    if (gi < ngrp) {
      const int F = grp ? grp[gi] : gi;
      s_t[i >> 5][i & 31] = lv0.tbar[4 * (size_t)(8 * F) + (i & 31)];
    }
  }
  __syncthreads();
  for (int i = t; i < GB * 32; i += 256) {
    const int gl = i >> 5, q = (i >> 3) & 3, pi = i & 7;
    if (g0 + gl >= ngrp) continue;
    double y = 0.0;
    for (int o = 0; o < 8; ++o) y += parity_sign(pi, o) * s_t[gl][4 * o + q];
    sY[gl][q][pi] = y;
  }
  __syncthreads();
  const double* w7 = l2p + (size_t)7 * 4 * K;
  for (int i = t; i < GB * K; i += 256) {
    const int gl = i / K, b = i - gl * K;
    if (g0 + gl >= ngrp) continue;
    const int F = grp ? grp[g0 + gl] : g0 + gl;
    const int par = (mi[4 * b] & 1) | (mi[4 * b + 1] & 1) << 1 | (mi[4 * b + 2] & 1) << 2;
    double acc = w7[b] * sY[gl][0][par];
    for (int c = 0; c < 3; ++c) acc += w7[(size_t)(1 + c) * K + b] * sY[gl][1 + c][par ^ (1 << c)];
    lv1.lbar[(size_t)F * K + b] += acc;
  }
}

// L2L^T over the M2L groups F of level f-1 (refined cells with a refined
// child): L_bar[F]_c += sum over the refined children y_o of
// 2^(-1-|b|) u_o^(c-b)/(c-b)! L_bar[y_o]_b, b <= c.  The child offsets u_o
// have components +-1/4, so the weight of child o is that of child 7 times
// (-1)^popcount(~o & q), q the parity of c - b: thread (group, b) first folds
// the 8 children's bars into Z_q[b] = sum_o (-1)^popcount(~o & q) L_bar[y_o]_b
// (a Walsh-Hadamard butterfly), then thread (group, c) sums the (b, c - b)
// entries of c (cm.l2lT_*, one weight each) against Z.  GB groups per block.
template <int P>
__global__ __launch_bounds__(256) void k_adj_l2l(const int32_t* __restrict__ grp, int ngrp, LevelDev lv1,
                                                 LevelDev lv0, CommonDev cm) {
  constexpr int K = nmi(P);
  constexpr int GB = 256 / K;
  __shared__ double sZ[GB][8][K];
  __shared__ int sR[GB][8];
  const int t = threadIdx.x;
  for (int i = t; i < GB * 8; i += 256) {
    const int gj = blockIdx.x * GB + (i >> 3);
    sR[i >> 3][i & 7] = gj < ngrp ? lv0.rank[8 * grp[gj] + (i & 7)] : -1;
  }
  __syncthreads();
  const int gl = t / K, b = t - gl * K;
  const int gi = blockIdx.x * GB + gl;
  const bool active = gl < GB && gi < ngrp;
  if (active) {
    // w[x] = bar of child 7 - x; after the butterfly w[q] = sum_x (-1)^popcount(x & q) w[x]
    double w[8];
#pragma unroll
    for (int x = 0; x < 8; ++x) {
      const int r = sR[gl][7 - x];
      w[x] = r >= 0 ? lv0.lbar[(size_t)r * K + b] : 0.0;
    }
#pragma unroll
    for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
      for (int x = 0; x < 8; ++x)
        if (!(x & bit)) {
          const double u = w[x], v = w[x | bit];
          w[x] = u + v;
          w[x | bit] = u - v;
        }
#pragma unroll
    for (int q = 0; q < 8; ++q) sZ[gl][q][b] = w[q];
  }
  __syncthreads();
  if (!active) return;
  const int c = b;
  double acc = 0.0;
  for (int j = cm.l2lT_start[c]; j < cm.l2lT_start[c + 1]; ++j) {
    const int code = cm.l2lT_list[j];
    acc += cm.l2lT_w[j] * sZ[gl][(code >> 24) & 7][code & 255];
  }
  lv1.lbar[(size_t)grp[gi] * K + c] += acc;
}

// M2M^T into the leaf children of the refined cells of level l-1: the
// monopole entry of every coefficient, folded per parity class first
// (Y_q = sum over a of parity q of w_a S_bar_a), then m_bar(o) += sum_q sign_q(o) Y_q.
// Block = kLeafupParents parents (rows staged in LDS), thread = (parent, parity
// class), then thread = (parent, child octant).
constexpr int kLeafupParents = 32;

template <int P>
__global__ __launch_bounds__(256) void k_adj_leafup(LevelDev lv1, LevelDev lv0, CommonDev cm) {
  constexpr int K = nmi(P);
  constexpr int NPB = kLeafupParents;
  __shared__ double sS[NPB * K];
  __shared__ double sY[NPB][8];
  const int t = threadIdx.x;
  const int r0 = blockIdx.x * NPB;
  const int np = min(NPB, lv1.nref - r0);
  for (int i = t; i < np * K; i += 256) sS[i] = lv1.sbar[(size_t)r0 * K + i];
  __syncthreads();
  const int j = t >> 3, q = t & 7;
  if (j < np) {
    double y = 0.0;
    for (int e = cm.m2mT_start[0]; e < cm.m2mT_start[1]; ++e) {
      const int code = cm.m2mT_list[e];
      if ((code >> 12) == q) y += cm.m2mT_w[e] * sS[j * K + (code & 4095)];
    }
    sY[j][q] = y;
  }
  __syncthreads();
  if (j < np) {
    const int o = q, c = 8 * (r0 + j) + o;
    if (lv0.rank[c] < 0) {
      double v = 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u) v += parity_sign(u, o) * sY[j][u];
      lv0.mbar[c] += v;
    }
  }
}

// Source-copy bars -> multipole bars, and M2M^T from the parent (levels
// processed coarse to fine): S_bar[r]_k = c_k 2^|k| Sc_bar[r]_k
//   + sum over the M2M entries (a, k, parity q) of w sign_q(o_r) S_bar[parent]_a.
// Over the refined parents at level f-1 that have a refined child (list grp):
// a block stages the entry lists once, then takes GB parents at a time (rows
// in LDS) with thread = (parent, k): one pass over the entries of k updates
// coefficient k of all 8 children.  Without a parent (f = 2) only the scaling
// (k_adj_scale).
template <int P>
__global__ __launch_bounds__(256) void k_adj_down(const int32_t* __restrict__ grp, int ngrp, LevelDev lv1,
                                                  LevelDev lv0, CommonDev cm) {
  constexpr int K = nmi(P);
  constexpr int NE = nmi_entries(P);
  constexpr int GB = 256 / K > 0 ? 256 / K : 1;
  __shared__ double sP[GB][K];
  __shared__ int sR[GB][8];
  __shared__ int sStart[K + 1];
  __shared__ int sList[NE];
  __shared__ double sW[NE];
  const int t = threadIdx.x;
  for (int i = t; i <= K; i += 256) sStart[i] = cm.m2mT_start[i];
  for (int i = t; i < NE; i += 256) {
    sList[i] = cm.m2mT_list[i];
    sW[i] = cm.m2mT_w[i];
  }
  const int gl = t / K, k = t - gl * K;
  for (int g0 = blockIdx.x * GB; g0 < ngrp; g0 += gridDim.x * GB) {
    __syncthreads();  // tables staged; the previous round is done with sP and sR
    for (int i = t; i < GB * 8; i += 256) {
      const int gi = g0 + (i >> 3);
      sR[i >> 3][i & 7] = gi < ngrp ? lv0.rank[8 * (size_t)grp[gi] + (i & 7)] : -1;
    }
    for (int i = t; i < GB * K; i += 256) {
      const int gj = i / K, gi = g0 + gj;
      if (gi < ngrp) sP[gj][i - gj * K] = lv1.sbar[(size_t)grp[gi] * K + (i - gj * K)];
    }
    __syncthreads();
    if (gl >= GB || g0 + gl >= ngrp) continue;
    double v[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      const int rc = sR[gl][o];
      v[o] = rc >= 0 ? cm.cfac2[k] * lv0.sbar[(size_t)rc * K + k] : 0.0;
    }
    for (int e = sStart[k]; e < sStart[k + 1]; ++e) {
      const int code = sList[e];
      const double w = sW[e], sp = sP[gl][code & 4095];
      const int q = code >> 12;
#pragma unroll
      for (int o = 0; o < 8; ++o) v[o] += w * parity_sign(q, o) * sp;
    }
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      const int rc = sR[gl][o];
      if (rc >= 0) lv0.sbar[(size_t)rc * K + k] = v[o];
    }
  }
}

template <int P>
__global__ void k_adj_scale(LevelDev lv0, CommonDev cm) {
  constexpr int K = nmi(P);
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= lv0.nref * K) return;
  lv0.sbar[i] *= cm.cfac2[i % K];
}

// Mass bars to the caller's slots: leaf cells of rebuilt levels get their bar
// (plus the transpose of the optional self term: the unit-form potential of a
// target holds -cself m, so its bar adds -cself T_phi), every other slot of
// the level gets 0.
__global__ void k_adj_out(LevelDev lv0, int rebuilt, double cself, double* __restrict__ mbar_out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= lv0.n) return;
  const int s = lv0.slot[c];
  if (s < 0) return;
  mbar_out[s] = (rebuilt && lv0.rank[c] < 0) ? lv0.mbar[c] - cself * lv0.tbar[4 * (size_t)c] : 0.0;
}

// ---------------------------------------------------------------------------
// MFMA forms of the transposed M2P and M2L.  A tile = 16 source cells of one
// octant class at level ls; for each of the 189 transposed taps the tap's
// group F of every column is found through the column's parent neighbours,
// and the contribution of F's 8 children (targets) is a dense product
//   OUT[K rows a x 16 columns] += A[K x k] * B[k x 16]
// with the D~ rows of the tap's offset staged in LDS (A read through per-lane
// offsets) and B loaded straight into registers.  One wave per block; each
// source cell belongs to one tile, so its bars have one writer.

// Unit-form target bars of the leaf children of every group at level ls, as
// the B operand of the transposed M2P: tbT[F][4 o + q] = T_(8F+o) with the
// acceleration bars negated (the forward M2P stores -acc), in T.
template <typename T>
__global__ void k_adj_tbT(LevelDev lvs, LevelDev lvt, T* __restrict__ tbT) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= lvs.nref * 32) return;
  const int F = i >> 5, j = i & 31;
  const double v = lvt.tbar[4 * (size_t)(8 * F) + j];
  tbT[i] = (T)((j & 3) == 0 ? v : -v);
}

// Local-expansion bars of level f in T and in the lane-group layout of the
// source copies (coefficient b at src_pos(b), zero padded).
template <typename T, int P>
__global__ void k_adj_lbarT(LevelDev lv, T* __restrict__ lT) {
  constexpr int K = nmi(P), STP = src_stp(P, (int)sizeof(T)), ROW = 4 * STP;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= lv.nref * ROW) return;
  const int r = i / ROW, b = i - r * ROW;   // b runs over coefficient indices 0 .. ROW-1
  lT[(size_t)r * ROW + src_pos(b, (int)sizeof(T))] = b < K ? (T)lv.lbar[(size_t)r * K + b] : (T)0;
}

// Per-block setup shared by both kernels: the 16 source cells, the child base
// (8 x refined rank, level ls) of each column's parent neighbours, the class
// taps.  Returns the octant class.
__device__ inline void adj_tile_setup(const int32_t* __restrict__ rec, const LevelDev& lvp, int* sS, int* sCB,
                                      int* sTap, const int32_t* __restrict__ tapsT) {
  const int lane = threadIdx.x;
  if (lane < 16) sS[lane] = rec[1 + lane];
  __syncthreads();
  for (int i = lane; i < 16 * 27; i += 64) {
    const int n = i / 27, e = i - n * 27;
    const int c = sS[n];
    int v = -1;
    if (c >= 0) {
      const int Q = lvp.nbr[(size_t)(c >> 3) * 27 + e];
      if (Q >= 0) {
        const int rQ = lvp.rank[Q];
        if (rQ >= 0) v = 8 * rQ;
      }
    }
    sCB[i] = v;
  }
  const int os = sS[0] & 7;
  for (int i = lane; i < kTapsT; i += 64) sTap[i] = tapsT[os * kTapsT + i];
}

// group (refined rank at level ls) of column n for transposed tap `code`, or -1
__device__ inline int adj_group(int code, int n, const int* sCB, const int32_t* __restrict__ rank_s) {
  const int cb = sCB[n * 27 + (code & 31)];
  return cb < 0 ? -1 : rank_s[cb + ((code >> 5) & 7)];
}

// Work item of this workgroup in its XCD's range, or -1.
__device__ inline int xcd_item(const XcdRanges& xr) {
  const int x = (int)(blockIdx.x & 7), item = xr.start[x] + (int)(blockIdx.x >> 3);
  return item < xr.start[x + 1] ? item : -1;
}

// Taps of [tb, te) whose group has a target child in at least one of the 16
// columns, moved in tap order to the front of sTap (one wave: lane group g
// tests tap i0 + g; a tap is written at an index no larger than its own, after
// every lane has read it); returns their number.  The other taps add nothing
// (every B is zero).
__device__ inline int adj_live_taps(int tb, int te, int* sTap, const int* sCB, const int32_t* __restrict__ rank_s,
                                    const uint8_t* __restrict__ live) {
  const int lane = threadIdx.x, n = lane & 15, g = lane >> 4;
  int cnt = 0;
  for (int i0 = tb; i0 < te; i0 += 4) {
    bool hit = false;
    if (i0 + g < te) {
      const int rF = adj_group(sTap[i0 + g], n, sCB, rank_s);
      hit = rF >= 0 && live[rF] != 0;
    }
    const uint64_t m = __ballot(hit);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if ((m >> (16 * j)) & 0xffffull) {
        if (lane == 0) sTap[cnt] = sTap[i0 + j];
        ++cnt;
      }
  }
  __syncthreads();
  return cnt;
}

// Output rows of one 16-row tile: multipole-source bars of refined sources,
// the monopole row of leaf sources into their mass bars; with a tap split,
// the rows go to the block's partial set part[(chunk * ntiles + tile) * 16 + n][K]
// instead, summed in order by k_adj_reduce.
template <typename T, int K>
__device__ inline void adj_write(const typename Acc4<T>::type& acc, int rt, int lane, int s, const LevelDev& lvs,
                                 double* part) {
  if (s < 0) return;
  if (part) {
    const int krow = lane >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = 16 * rt + acc_row<T>(krow, r);
      if (a < K) part[(size_t)(lane & 15) * K + a] = (double)acc[r];
    }
    return;
  }
  const int rs = lvs.rank[s];
  const int krow = lane >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int a = 16 * rt + acc_row<T>(krow, r);
    if (rs >= 0) {
      if (a < K) lvs.sbar[(size_t)rs * K + a] += (double)acc[r];
    } else if (a == 0) {
      lvs.mbar[s] += (double)acc[r];
    }
  }
}

// Step kb of the transposed M2P carries quantity q = kb & 3 (phi, then the
// three acceleration components) of two children.  Multipole coefficients of
// order p enter the forward M2P only through the potential (the accelerations
// use orders < p), so a 16-row tile whose rows are all of order p has zero A
// entries in the acceleration steps: they are skipped (adding zeros would not
// change a bit of the result).
template <int P>
__host__ __device__ constexpr bool adj_m2p_step_used(int rt, int kb) {
  int d = 0;
  while (nmi(d) <= 16 * rt) ++d;  // order of the tile's first row
  return d < P || (kb & 3) == 0;
}

// Transposed intermediate-field M2P: targets = leaf children (level ls + 1) of
// the groups reading the source; k = (child o, quantity q) with lane group g
// holding j = 8 g + kb, so its B fragments are 8 consecutive values of tbT.
template <typename T, int P>
__global__ __launch_bounds__(64) void k_adj_m2p_mfma(const int32_t* __restrict__ tiles, XcdRanges xr, int nsplit,
                                                     double* __restrict__ part, const int32_t* __restrict__ tapsT,
                                                     const uint8_t* __restrict__ live,
                                                     const int16_t* __restrict__ aoff, LevelDev lvp, LevelDev lvs,
                                                     const T* __restrict__ tbT, const T* __restrict__ Dst) {
  constexpr int K = nmi(P), RT = (K + 15) / 16;
  constexpr int SDP = dstage_len(P, (int)sizeof(T));
  constexpr int VW = 16 / (int)sizeof(T), NVB = 8 / VW, ND = (SDP / VW + 63) / 64;
  using V = typename Vec16<T>::type;
  __shared__ __align__(16) T sD[2][SDP];
  __shared__ int sS[16];
  __shared__ int sCB[16 * 27];
  __shared__ int sTap[kTapsT];
  const int item = xcd_item(xr);
  if (item < 0) return;
  const int ntiles = xr.start[8] / nsplit;
  const int tile = item / nsplit, chunk = item - tile * nsplit;
  const int tb = chunk * kTapsT / nsplit, te = (chunk + 1) * kTapsT / nsplit;
  const int lane = threadIdx.x, n = lane & 15, g = lane >> 4;
  adj_tile_setup(tiles + (size_t)tile * 17, lvp, sS, sCB, sTap, tapsT);
  int off[RT][8];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int kb = 0; kb < 8; ++kb) off[rt][kb] = aoff[(rt * 8 + kb) * 64 + lane];
  __syncthreads();
  const int nt = adj_live_taps(tb, te, sTap, sCB, lvs.rank, live);
  gptr<T> tbTg = as_global(tbT);
  auto loadB = [&](int rF, V* b) {
    if (rF >= 0) {
      gptr<V> src = (gptr<V>)(tbTg + (size_t)rF * 32 + 8 * g);
#pragma unroll
      for (int j = 0; j < NVB; ++j) b[j] = src[j];
    } else {
#pragma unroll
      for (int j = 0; j < NVB; ++j) b[j] = V{};
    }
  };
  typename Acc4<T>::type acc[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) acc[rt] = {0, 0, 0, 0};
  if (nt > 0) {
    V bA[NVB], bB[NVB];
    V vD[ND];
    int gn = adj_group(sTap[0], n, sCB, lvs.rank);
    loadB(gn, bA);
    load_dstage_t<T, SDP, 64>(sTap[0] >> 8, Dst, vD);
    // both buffers hold finite rows from the start (the empty tap below reads one)
    store_dstage_t<T, SDP, 64>(sD[0], vD);
    store_dstage_t<T, SDP, 64>(sD[1], vD);
    gn = adj_group(sTap[1 < nt ? 1 : 0], n, sCB, lvs.rank);
    __syncthreads();
    // Taps run in pairs; an odd count ends with one empty tap (B zero), so
    // that both steps of a pair run unconditionally (no accumulator moves
    // between them).
    const int nt2 = (nt + 1) & ~1;
    auto step = [&](int k, int b, const V* bc, V* bn) {
      const int k1 = k + 1 < nt ? k + 1 : nt - 1;
      loadB(k + 1 < nt ? gn : -1, bn);
      load_dstage_t<T, SDP, 64>(sTap[k1] >> 8, Dst, vD);
      gn = adj_group(sTap[k + 2 < nt ? k + 2 : nt - 1], n, sCB, lvs.rank);
      const T* D = sD[b];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int kb = 0; kb < 8; ++kb)
          if (adj_m2p_step_used<P>(rt, kb)) acc[rt] = mfma16(D[off[rt][kb]], bc[kb / VW][kb % VW], acc[rt]);
      store_dstage_t<T, SDP, 64>(sD[b ^ 1], vD);
      __syncthreads();
    };
    for (int k = 0; k < nt2; k += 2) {
      step(k, 0, bA, bB);
      step(k + 1, 1, bB, bA);
    }
  }
  const int s = sS[n];
  double* pp = nsplit > 1 ? part + ((size_t)chunk * ntiles + tile) * 16 * K : nullptr;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) adj_write<T, K>(acc[rt], rt, lane, s, lvs, pp);
}

// Transposed M2L: targets = refined children y (level ls + 1) of the groups
// reading the source; for each tap and child octant o, A = D~_(a+b)(R~_o)
// (triangle |a| + |b| <= p skipped at k-step granularity) and B = the local-
// expansion bars of child o, b = 4 kb + g from the lane-group layout.
template <int P>
struct AdjM2LPlan {
  static constexpr int RT = (nmi(P) + 15) / 16;
  int ks[RT] = {};
  int base[RT] = {};
  int total = 0;
  int kbmax = 0;
};
template <int P>
constexpr AdjM2LPlan<P> make_adj_m2l_plan() {
  AdjM2LPlan<P> pl{};
  for (int rt = 0; rt < AdjM2LPlan<P>::RT; ++rt) {
    int d = 0;
    while (nmi(d) <= 16 * rt) ++d;  // degree of the tile's first row
    pl.ks[rt] = (nmi(P - d) + 3) / 4;
    pl.base[rt] = pl.total;
    pl.total += pl.ks[rt];
    if (pl.ks[rt] > pl.kbmax) pl.kbmax = pl.ks[rt];
  }
  return pl;
}

template <typename T, int P>
__global__ __launch_bounds__(64) void k_adj_m2l_mfma(const int32_t* __restrict__ tiles, XcdRanges xr, int nsplit,
                                                     double* __restrict__ part, const int32_t* __restrict__ tapsT,
                                                     const uint8_t* __restrict__ live,
                                                     const int16_t* __restrict__ aoff, LevelDev lvp, LevelDev lvs,
                                                     LevelDev lvt, const T* __restrict__ lT,
                                                     const T* __restrict__ Dst) {
  constexpr int K = nmi(P), KS = dstage_ks(P), SDP = dstage_len(P, (int)sizeof(T));
  constexpr AdjM2LPlan<P> PL = make_adj_m2l_plan<P>();
  constexpr int RT = AdjM2LPlan<P>::RT;
  constexpr int VW = 16 / (int)sizeof(T), STP = src_stp(P, (int)sizeof(T)), ROW = 4 * STP;
  constexpr int NVB = (PL.kbmax + VW - 1) / VW, ND = (SDP / VW + 63) / 64;
  using V = typename Vec16<T>::type;
  __shared__ __align__(16) T sD[2][SDP];
  __shared__ int sS[16];
  __shared__ int sCB[16 * 27];
  __shared__ int sTap[kTapsT];
  const int item = xcd_item(xr);
  if (item < 0) return;
  const int ntiles = xr.start[8] / nsplit;
  const int tile = item / nsplit, chunk = item - tile * nsplit;
  const int tb = chunk * kTapsT / nsplit, te = (chunk + 1) * kTapsT / nsplit;
  const int lane = threadIdx.x, n = lane & 15, g = lane >> 4;
  adj_tile_setup(tiles + (size_t)tile * 17, lvp, sS, sCB, sTap, tapsT);
  int off[PL.total];
#pragma unroll
  for (int i = 0; i < PL.total; ++i) off[i] = aoff[i * 64 + lane];
  __syncthreads();
  const int nt = adj_live_taps(tb, te, sTap, sCB, lvs.rank, live);
  // Local-expansion-bar rows (refined ranks at level ls + 1) of the 8 children
  // of a tap's group: loaded together one tap ahead, so that the B loads of a
  // sub-step never wait for a rank.  Loads go through global-address pointers
  // (flat loads would also count against the wait for the LDS A reads).
  gptr<int32_t> rankt = as_global(lvt.rank);
  gptr<T> lTg = as_global(lT);
  auto children = [&](int rF, int* ry) {
#pragma unroll
    for (int o = 0; o < 8; ++o) ry[o] = rankt[8 * (rF >= 0 ? rF : 0) + o];
#pragma unroll
    for (int o = 0; o < 8; ++o) ry[o] = rF >= 0 ? ry[o] : -1;
  };
  auto loadB = [&](int ry, V* b) {
    if (ry >= 0) {
      gptr<T> src = lTg + (size_t)ry * ROW;
#pragma unroll
      for (int j = 0; j < NVB; ++j) b[j] = *(gptr<V>)(src + src_vec(j, g, (int)sizeof(T)));
    } else {
#pragma unroll
      for (int j = 0; j < NVB; ++j) b[j] = V{};
    }
  };
  typename Acc4<T>::type acc[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) acc[rt] = {0, 0, 0, 0};
  if (nt > 0) {
    V bA[NVB], bB[NVB];
    V vD[ND];
    int ryc[8], ryn[8];
    int gnext = 1 < nt ? adj_group(sTap[1], n, sCB, lvs.rank) : -1;
    children(adj_group(sTap[0], n, sCB, lvs.rank), ryc);
    children(gnext, ryn);
    loadB(ryc[0], bA);
    load_dstage_t<T, SDP, 64>(sTap[0] >> 8, Dst, vD);
    store_dstage_t<T, SDP, 64>(sD[0], vD);
    __syncthreads();
    // sub-step (tap k, octant o): B of (k, o) in bc; prefetch (k, o+1) or (k+1, 0) into bn
    auto sub = [&](int k, int o, const V* bc, V* bn) {
      const int b = k & 1;
      if (o < 7) loadB(ryc[o + 1], bn);
      else if (k + 1 < nt) loadB(ryn[0], bn);
      const T* D = sD[b] + o * KS;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int kb = 0; kb < PL.ks[rt]; ++kb)
          acc[rt] = mfma16(D[off[PL.base[rt] + kb]], bc[kb / VW][kb % VW], acc[rt]);
    };
    for (int k = 0; k < nt; ++k) {
      const int b = k & 1;
      if (k + 1 < nt) load_dstage_t<T, SDP, 64>(sTap[k + 1] >> 8, Dst, vD);
#pragma unroll
      for (int o = 0; o < 8; o += 2) {
        sub(k, o, bA, bB);
        sub(k, o + 1, bB, bA);
      }
      if (k + 1 < nt) store_dstage_t<T, SDP, 64>(sD[b ^ 1], vD);
#pragma unroll
      for (int o = 0; o < 8; ++o) ryc[o] = ryn[o];
      if (k + 2 < nt) {
        gnext = adj_group(sTap[k + 2], n, sCB, lvs.rank);
        children(gnext, ryn);
      }
      __syncthreads();
    }
  }
  const int s = sS[n];
  double* pp = nsplit > 1 ? part + ((size_t)chunk * ntiles + tile) * 16 * K : nullptr;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) adj_write<T, K>(acc[rt], rt, lane, s, lvs, pp);
}

// Ordered sum of the tap-split partial sets of a transposed translation into
// the source bars (thread = tile column x coefficient).
template <int P>
__global__ void k_adj_reduce(const int32_t* __restrict__ tiles, int ntiles, int nsplit,
                             const double* __restrict__ part, LevelDev lvs) {
  constexpr int K = nmi(P);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntiles * 16 * K) return;
  const int col = i / K, a = i - col * K;
  const int s = tiles[(size_t)(col >> 4) * 17 + 1 + (col & 15)];
  if (s < 0) return;
  const int rs = lvs.rank[s];
  if (rs < 0 && a != 0) return;
  double v = 0.0;
  for (int c = 0; c < nsplit; ++c) v += part[((size_t)c * ntiles * 16 + col) * K + a];
  if (rs >= 0) lvs.sbar[(size_t)rs * K + a] += v;
  else lvs.mbar[s] += v;
}

// ---------------------------------------------------------------------------
// launchers

#define AFMM_P_SWITCH(p, X) \
  switch (p) {              \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) default : return hipErrorInvalidValue; \
  }

hipError_t launch_adj_init(const LevelDev& lv, int target, const double* phib, const double* accb, double sp,
                           double sa, hipStream_t st) {
  if (lv.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_init, dim3((lv.n + 255) / 256), dim3(256), 0, st, lv.n, lv.rank, lv.slot, target, phib,
                     accb, sp, sa, lv.tbar, lv.mbar);
  return hipGetLastError();
}

hipError_t launch_adj_zero(double* p, size_t n, hipStream_t st) {
  if (n == 0 || !p) return hipSuccess;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_adj_zero, dim3((unsigned)blocks), dim3(256), 0, st, n, p);
  return hipGetLastError();
}

hipError_t launch_adj_near(int p, const int32_t* leafgrp, int nleafgrp, const int32_t* vgrp, int nvgrp,
                           const int32_t* refgrp, int nrefgrp, const LevelDev& lv1, const LevelDev& lv0,
                           const LevelDev& lvp, int targets_here, const TablesDev<double>& t64, const CommonDev& cm,
                           hipStream_t st) {
  if (lv1.nref == 0) return hipSuccess;
  if (targets_here && nleafgrp > 0) {
    const int ntiles = (nleafgrp + 15) / 16;
    hipLaunchKernelGGL(k_adj_near_mfma, dim3(8 * ((ntiles + 7) / 8)), dim3(256), 0, st, leafgrp, nleafgrp, lv1, lv0,
                       t64.adjNearA);
  }
  if (nvgrp > 0) hipLaunchKernelGGL(k_adj_near_leaf, dim3(nvgrp), dim3(256), 0, st, vgrp, lv1, lv0, lvp);
  if (!targets_here || !lv0.sbar || nrefgrp == 0) return hipGetLastError();
  // refgrp == nullptr: every refined cell of level l-1
  const int nb = refgrp ? nrefgrp : lv1.nref;
#define X(PP)                                                                                                  \
  case PP:                                                                                                     \
    hipLaunchKernelGGL((k_adj_near_m2p<PP>), dim3(nb), dim3(256), 0, st, refgrp, lv1, lv0, t64.Dsame, t64.cfacn, \
                       cm.up);                                                                                 \
    break;
  AFMM_P_SWITCH(p, X)
#undef X
  return hipGetLastError();
}

hipError_t launch_adj_l2p(int p, const int32_t* grp, int ngrp, const LevelDev& lv1, const LevelDev& lv0,
                          const TablesDev<double>& t64, const CommonDev& cm, hipStream_t st) {
  if (ngrp == 0) return hipSuccess;
  const int gb = std::max(256 / nmi(p), 1);
#define X(PP)                                                                                              \
  case PP:                                                                                                 \
    hipLaunchKernelGGL((k_adj_l2p<PP>), dim3((ngrp + gb - 1) / gb), dim3(256), 0, st, grp, ngrp, lv1, lv0, \
                       t64.l2p, cm.mi);                                                                    \
    break;
  AFMM_P_SWITCH(p, X)
#undef X
  return hipGetLastError();
}

hipError_t launch_adj_l2l(int p, const int32_t* grp, int ngrp, const LevelDev& lv1, const LevelDev& lv0,
                          const TablesDev<double>& t64, const CommonDev& cm, hipStream_t st) {
  (void)t64;
  if (ngrp == 0) return hipSuccess;
  const int gb = 256 / nmi(p);
#define X(PP)                                                                                                  \
  case PP:                                                                                                     \
    hipLaunchKernelGGL((k_adj_l2l<PP>), dim3((ngrp + gb - 1) / gb), dim3(256), 0, st, grp, ngrp, lv1, lv0, cm); \
    break;
  AFMM_P_SWITCH(p, X)
#undef X
  return hipGetLastError();
}

hipError_t launch_adj_down(int p, const int32_t* grp, int ngrp, const LevelDev& lv1, const LevelDev& lv0,
                           int has_parent, const CommonDev& cm, hipStream_t st) {
  const int n = lv0.nref * nmi(p);
  if (n == 0) return hipSuccess;
  if (has_parent) {
    if (ngrp == 0) return hipSuccess;
    if (!grp) return hipErrorInvalidValue;
    const int gb = std::max(256 / nmi(p), 1);
    const int blocks = std::min((ngrp + gb - 1) / gb, 2048);
#define X(PP)                                                                                                       \
  case PP:                                                                                                          \
    hipLaunchKernelGGL((k_adj_down<PP>), dim3(blocks), dim3(256), 0, st, grp, ngrp, lv1, lv0, cm);                \
    break;
    AFMM_P_SWITCH(p, X)
#undef X
  } else {
#define X(PP) \
  case PP: hipLaunchKernelGGL((k_adj_scale<PP>), dim3((n + 255) / 256), dim3(256), 0, st, lv0, cm); break;
    AFMM_P_SWITCH(p, X)
#undef X
  }
  return hipGetLastError();
}

hipError_t launch_adj_out(int p, const LevelDev& lv1, const LevelDev& lv0, int has_parent, int rebuilt,
                          double cself, const CommonDev& cm, double* mbar_out, hipStream_t st) {
  if (lv0.n == 0) return hipSuccess;
  if (has_parent && lv1.nref > 0) {
#define X(PP) \
  case PP: hipLaunchKernelGGL((k_adj_leafup<PP>), dim3((lv1.nref + kLeafupParents - 1) / kLeafupParents), dim3(256), 0, st, lv1, lv0, cm); break;
    AFMM_P_SWITCH(p, X)
#undef X
  }
  hipLaunchKernelGGL(k_adj_out, dim3((lv0.n + 255) / 256), dim3(256), 0, st, lv0, rebuilt, cself, mbar_out);
  return hipGetLastError();
}

static hipError_t adj_reduce(int p, const int32_t* tiles, int ntiles, int nsplit, const double* part,
                             const LevelDev& lvs, hipStream_t st) {
  if (nsplit <= 1) return hipGetLastError();
  const int n = ntiles * 16 * nmi(p);
#define X(PP) \
  case PP: hipLaunchKernelGGL((k_adj_reduce<PP>), dim3((n + 255) / 256), dim3(256), 0, st, tiles, ntiles, nsplit, part, lvs); break;
  AFMM_P_SWITCH(p, X)
#undef X
  return hipGetLastError();
}

template <typename T>
static hipError_t adj_m2p_t(int p, const int32_t* tiles, int ntiles, int nsplit, const XcdRanges& xr,
                            const uint8_t* live, double* part,
                            const int32_t* tapsT,
                            const int16_t* aoff, const LevelDev& lvp, const LevelDev& lvs, const LevelDev& lvt,
                            const T* Dst, hipStream_t st) {
  T* tbT = (T*)lvs.tbT;
  hipLaunchKernelGGL((k_adj_tbT<T>), dim3((lvs.nref * 32 + 255) / 256), dim3(256), 0, st, lvs, lvt, tbT);
  if (xr.start[8] != ntiles * nsplit) return hipErrorInvalidValue;
  const dim3 grid(xr.grid()), block(64);
#define X(PP) \
  case PP: hipLaunchKernelGGL((k_adj_m2p_mfma<T, PP>), grid, block, 0, st, tiles, xr, nsplit, part, tapsT, live, aoff, lvp, lvs, (const T*)tbT, Dst); break;
  AFMM_P_SWITCH(p, X)
#undef X
  return adj_reduce(p, tiles, ntiles, nsplit, part, lvs, st);
}

hipError_t launch_adj_m2p_mfma(int p, bool fp32, const int32_t* tiles, int ntiles, int nsplit, const XcdRanges& xr,
                               const uint8_t* live, double* part, const int32_t* tapsT, const int16_t* aoff, const LevelDev& lvp,
                               const LevelDev& lvs, const LevelDev& lvt, const TablesDev<float>& t32,
                               const TablesDev<double>& t64, hipStream_t st) {
  if (ntiles <= 0 || lvs.nref == 0) return hipSuccess;
  if (!live) return hipErrorInvalidValue;
  if (fp32) return adj_m2p_t<float>(p, tiles, ntiles, nsplit, xr, live, part, tapsT, aoff, lvp, lvs, lvt, t32.Dstage, st);
  return adj_m2p_t<double>(p, tiles, ntiles, nsplit, xr, live, part, tapsT, aoff, lvp, lvs, lvt, t64.Dstage, st);
}

template <typename T>
static hipError_t adj_m2l_t(int p, const int32_t* tiles, int ntiles, int nsplit, const XcdRanges& xr,
                            const uint8_t* live, double* part,
                            const int32_t* tapsT,
                            const int16_t* aoff, const LevelDev& lvp, const LevelDev& lvs, const LevelDev& lvt,
                            const T* Dst, hipStream_t st) {
  T* lT = (T*)lvt.lbarT;
  const int rows = lvt.nref * src_row(p, (int)sizeof(T));
#define X(PP) \
  case PP: hipLaunchKernelGGL((k_adj_lbarT<T, PP>), dim3((rows + 255) / 256), dim3(256), 0, st, lvt, lT); break;
  AFMM_P_SWITCH(p, X)
#undef X
  if (xr.start[8] != ntiles * nsplit) return hipErrorInvalidValue;
  const dim3 grid(xr.grid()), block(64);
#define X(PP) \
  case PP: hipLaunchKernelGGL((k_adj_m2l_mfma<T, PP>), grid, block, 0, st, tiles, xr, nsplit, part, tapsT, live, aoff, lvp, lvs, lvt, (const T*)lT, Dst); break;
  AFMM_P_SWITCH(p, X)
#undef X
  return adj_reduce(p, tiles, ntiles, nsplit, part, lvs, st);
}

hipError_t launch_adj_m2l_mfma(int p, bool fp32, const int32_t* tiles, int ntiles, int nsplit, const XcdRanges& xr,
                               const uint8_t* live, double* part, const int32_t* tapsT, const int16_t* aoff, const LevelDev& lvp,
                               const LevelDev& lvs, const LevelDev& lvt, const TablesDev<float>& t32,
                               const TablesDev<double>& t64, hipStream_t st) {
  if (ntiles <= 0 || lvt.nref == 0) return hipSuccess;
  if (!live) return hipErrorInvalidValue;
  if (fp32) return adj_m2l_t<float>(p, tiles, ntiles, nsplit, xr, live, part, tapsT, aoff, lvp, lvs, lvt, t32.Dstage, st);
  return adj_m2l_t<double>(p, tiles, ntiles, nsplit, xr, live, part, tapsT, aoff, lvp, lvs, lvt, t64.Dstage, st);
}

#undef AFMM_P_SWITCH

}  // namespace afmm
