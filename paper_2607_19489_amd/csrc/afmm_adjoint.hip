// Adjoint (transposed) pass of the adaptive FMM, FP64.
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
//   M2P, intermediate field                    M2P^T per source cell              k_adj_m2p
//   L2L (Eq. eq:L2L), top-down                 L2L^T, bottom-up                   k_adj_l2l
//   M2L (Eq. eq:M2L), 189-cell list            M2L^T per source cell              k_adj_m2l
//   source copy c_a 2^|a| S~_a                 scale of the source bar            k_adj_down
//   M2M (Eq. eq:M2M_general), bottom-up        M2M^T, top-down                    k_adj_down
//   mass gather (slot -> cell)                 scatter (cell -> slot)             k_adj_out
//
// Every relation is gathered from the receiving side, so no atomics are needed
// and the sums run in a fixed order.  The interaction list relation is
// symmetric at one level (s is in F's list iff |parent(s) - parent(F)| <= 1
// and |s - F| >= 2), so a source cell s finds every group F that reads it
// through its own parent's 27 neighbours: 189 "transposed taps" per octant of s.
#include <hip/hip_runtime.h>

#include "afmm_internal.h"

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

constexpr int threads_for(int K) { return ((K + 63) / 64) * 64; }

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

// P2P^T for the leaves s of level l (block = one refined cell F of level l-1,
// s = its child o).  Targets that read s through a P2P:
//   level l leaves n among the children of F's 27 neighbours (near field),
//   level l+1 children of a refined level-l n touching s (s is in their near
//     field as a coarse leaf),
//   level l-1 leaves q touching F (s is in q's nearest field).
__global__ __launch_bounds__(256) void k_adj_near_leaf(LevelDev lv1, LevelDev lv0, LevelDev lvp) {
  __shared__ int s_nb[27];
  __shared__ double s_red[256];
  const int F = blockIdx.x;
  const int t = threadIdx.x, o = t & 7, j = t >> 3;
  if (t < 27) s_nb[t] = lv1.nbr[(size_t)F * 27 + t];
  __syncthreads();
  const int s = 8 * F + o;
  double acc = 0.0;
  if (lv0.rank[s] < 0) {
    const int sx = ax_o(o, 0), sy = ax_o(o, 1), sz = ax_o(o, 2);
    for (int k = j; k < 216; k += 32) {
      const int e = k >> 3, op = k & 7;
      const int q = s_nb[e];
      if (q < 0) continue;
      const int ex = ax_e(e, 0), ey = ax_e(e, 1), ez = ax_e(e, 2);
      const int rq = lv1.rank[q];
      if (rq < 0) {
        // nearest field of the coarse leaf q = F + e: r = e - (o - 1/2)/2 in h_(l-1) units
        if (op == 0)
          acc += p2p_adj(ex - (sx - 0.5) * 0.5, ey - (sy - 0.5) * 0.5, ez - (sz - 0.5) * 0.5,
                         lv1.tbar + 4 * (size_t)q);
        continue;
      }
      const int n = 8 * rq + op;
      if (n == s) continue;
      const int tx = sx - 2 * ex - ax_o(op, 0), ty = sy - 2 * ey - ax_o(op, 1), tz = sz - 2 * ez - ax_o(op, 2);
      const int rn = lv0.rank[n];
      if (rn < 0) {
        acc += p2p_adj(-tx, -ty, -tz, lv0.tbar + 4 * (size_t)n);
      } else if (max(abs(tx), max(abs(ty), abs(tz))) <= 1) {
        for (int o2 = 0; o2 < 8; ++o2)
          acc += p2p_adj(ax_o(o2, 0) - 0.5 - 2.0 * tx, ax_o(o2, 1) - 0.5 - 2.0 * ty, ax_o(o2, 2) - 0.5 - 2.0 * tz,
                         lvp.tbar + 4 * (size_t)(8 * rn + o2));
      }
    }
  }
  s_red[t] = acc;
  __syncthreads();
  if (t < 8 && lv0.rank[8 * F + t] < 0) {
    double sum = 0.0;
    for (int jj = 0; jj < 32; ++jj) sum += s_red[t + 8 * jj];
    lv0.mbar[8 * F + t] += sum;
  }
}

// Near-field M2P^T: a refined level-l cell s is read, through 2^-|a| times its
// source copy, by the level-l leaves n among the children of F's neighbours
// that do not touch s.  Source-copy bar of s += cfacn_a (D_a T_phi - sum_i
// D_(a+e_i) T_i) with D = D~ at n - s.
template <int P>
__global__ __launch_bounds__(256) void k_adj_near_m2p(LevelDev lv1, LevelDev lv0, const double* __restrict__ Dsame,
                                                      const double* __restrict__ cfacn,
                                                      const int16_t* __restrict__ up) {
  constexpr int K = nmi(P), K1 = nmi(P - 1);
  __shared__ int s_cand[216];
  __shared__ int s_ref[8];
  const int F = blockIdx.x;
  const int t = threadIdx.x;
  if (t < 8) s_ref[t] = lv0.rank[8 * F + t];
  if (t < 216) {
    const int e = t >> 3, op = t & 7;
    const int q = lv1.nbr[(size_t)F * 27 + e];
    int v = -1;
    if (q >= 0) {
      const int rq = lv1.rank[q];
      if (rq >= 0 && lv0.rank[8 * rq + op] < 0) v = 8 * rq + op;
    }
    s_cand[t] = v;
  }
  __syncthreads();
  bool any = false;
  for (int o = 0; o < 8; ++o) any |= s_ref[o] >= 0;
  if (!any) return;
  for (int i = t; i < 8 * K; i += 256) {
    const int o = i / K, a = i - o * K;
    const int rs = s_ref[o];
    if (rs < 0) continue;
    double acc = 0.0;
    for (int k = 0; k < 216; ++k) {
      const int n = s_cand[k];
      if (n < 0) continue;
      const int e = k >> 3, op = k & 7;
      const int dx = 2 * ax_e(e, 0) + ax_o(op, 0) - ax_o(o, 0);
      const int dy = 2 * ax_e(e, 1) + ax_o(op, 1) - ax_o(o, 1);
      const int dz = 2 * ax_e(e, 2) + ax_o(op, 2) - ax_o(o, 2);
      if (max(abs(dx), max(abs(dy), abs(dz))) <= 1) continue;
      const double* D = Dsame + (size_t)dsame_index(dx, dy, dz) * K;
      const double* tb = lv0.tbar + 4 * (size_t)n;
      double v = D[a] * tb[0];
      if (a < K1) v -= D[up[3 * a + 0]] * tb[1] + D[up[3 * a + 1]] * tb[2] + D[up[3 * a + 2]] * tb[3];
      acc += v;
    }
    lv0.sbar[(size_t)rs * K + a] += cfacn[a] * acc;
  }
}

// L2P^T: the far field of the leaf children of F reads L~[F] (level l-1).
template <int P>
__global__ __launch_bounds__(256) void k_adj_l2p(LevelDev lv1, LevelDev lv0, const double* __restrict__ l2p) {
  constexpr int K = nmi(P);
  __shared__ double s_t[32];
  const int F = blockIdx.x;
  const int t = threadIdx.x;
  if (t < 32) s_t[t] = lv0.tbar[4 * (size_t)(8 * F) + t];
  __syncthreads();
  for (int b = t; b < K; b += 256) {
    double acc = 0.0;
    for (int o = 0; o < 8; ++o)
      for (int q = 0; q < 4; ++q) acc += l2p[((size_t)o * 4 + q) * K + b] * s_t[4 * o + q];
    lv1.lbar[(size_t)F * K + b] += acc;
  }
}

// Transposed-tap resolution for source cell s = 8 P + os at level l-1: the
// group F (refined rank at level l-1) and offset index of each tap, or -1.
__device__ inline void resolve_taps(int s, const LevelDev& lv2, const LevelDev& lv1, const int32_t* __restrict__ tapsT,
                                    int* sF, int* sDi) {
  const int os = s & 7, P = s >> 3;
  for (int i = threadIdx.x; i < kTapsT; i += blockDim.x) {
    const int code = tapsT[os * kTapsT + i];
    const int e = code & 31, oF = (code >> 5) & 7;
    int rF = -1;
    const int Q = lv2.nbr[(size_t)P * 27 + e];
    if (Q >= 0) {
      const int rQ = lv2.rank[Q];
      if (rQ >= 0) rF = lv1.rank[8 * rQ + oF];
    }
    sF[i] = rF;
    sDi[i] = code >> 8;
  }
}

// Intermediate-field M2P^T (block = one source cell s of level l-1): the leaf
// children c of every group F whose list holds s read c_a 2^|a| S~_a[s] (or
// the mass of a leaf s) with D~ at R~ = c - s.
template <int P>
__global__ __launch_bounds__(threads_for(nmi(P))) void k_adj_m2p(LevelDev lv2, LevelDev lv1, LevelDev lv0,
                                                                  const int32_t* __restrict__ tapsT,
                                                                  const double* __restrict__ Dil,
                                                                  const int16_t* __restrict__ up) {
  constexpr int K = nmi(P), K1 = nmi(P - 1), NT = threads_for(K);
  __shared__ int sF[kTapsT], sDi[kTapsT];
  __shared__ double sD[8 * K];
  __shared__ double sT[32];
  const int s = blockIdx.x;
  const int t = threadIdx.x;
  resolve_taps(s, lv2, lv1, tapsT, sF, sDi);
  const int rs = lv1.rank[s];
  double acc = 0.0;
  for (int i = 0; i < kTapsT; ++i) {
    __syncthreads();
    const int rF = sF[i];
    if (rF < 0) continue;
    const double* Dr = Dil + (size_t)sDi[i] * 8 * K;
    for (int k = t; k < 8 * K; k += NT) sD[k] = Dr[k];
    if (t < 32) sT[t] = lv0.tbar[4 * (size_t)(8 * rF) + t];
    __syncthreads();
    if (t < K && (rs >= 0 || t == 0)) {
      for (int o = 0; o < 8; ++o) {
        const double* D = sD + o * K;
        double v = D[t] * sT[4 * o];
        if (t < K1) v -= D[up[3 * t + 0]] * sT[4 * o + 1] + D[up[3 * t + 1]] * sT[4 * o + 2] +
                         D[up[3 * t + 2]] * sT[4 * o + 3];
        acc += v;
      }
    }
  }
  if (rs >= 0) {
    if (t < K) lv1.sbar[(size_t)rs * K + t] += acc;
  } else if (t == 0) {
    lv1.mbar[s] += acc;
  }
}

// L2L^T (block = one refined cell F of level f-1): L_bar[F]_c += sum over the
// refined children y and b <= c of 2^(-1-|b|) u^(c-b)/(c-b)! L_bar[y]_b.
template <int P>
__global__ __launch_bounds__(256) void k_adj_l2l(LevelDev lv1, LevelDev lv0, const double* __restrict__ l2lw,
                                                 const int8_t* __restrict__ mi) {
  constexpr int K = nmi(P);
  __shared__ double sL[8 * K];
  __shared__ int sR[8];
  const int F = blockIdx.x;
  const int t = threadIdx.x;
  if (t < 8) sR[t] = lv0.rank[8 * F + t];
  __syncthreads();
  for (int i = t; i < 8 * K; i += 256) {
    const int o = i / K, b = i - o * K;
    sL[i] = sR[o] >= 0 ? lv0.lbar[(size_t)sR[o] * K + b] : 0.0;
  }
  __syncthreads();
  for (int c = t; c < K; c += 256) {
    const int c0 = mi[4 * c], c1 = mi[4 * c + 1], c2 = mi[4 * c + 2];
    double acc = 0.0;
    for (int b = 0; b <= c; ++b) {
      const int g0 = c0 - mi[4 * b], g1 = c1 - mi[4 * b + 1], g2 = c2 - mi[4 * b + 2];
      if (g0 < 0 || g1 < 0 || g2 < 0) continue;
      const int g = mi_index(g0, g1, g2), nb = mi[4 * b + 3];
      for (int o = 0; o < 8; ++o) acc += l2lw[((size_t)o * (P + 1) + nb) * K + g] * sL[o * K + b];
    }
    lv1.lbar[(size_t)F * K + c] += acc;
  }
}

// M2L^T (block = one source cell s of level f-1): every refined child y of a
// group F whose list holds s reads c_a 2^|a| S~_a[s] through D~_(a+b)(R~),
// R~ = y - s, |a| + |b| <= p.
template <int P>
__global__ __launch_bounds__(threads_for(nmi(P))) void k_adj_m2l(LevelDev lv2, LevelDev lv1, LevelDev lv0,
                                                                  const int32_t* __restrict__ tapsT,
                                                                  const double* __restrict__ Dil,
                                                                  const int16_t* __restrict__ sumidx,
                                                                  const int8_t* __restrict__ mi) {
  constexpr int K = nmi(P), NT = threads_for(K);
  __shared__ int sF[kTapsT], sDi[kTapsT];
  __shared__ double sD[8 * K];
  __shared__ double sL[8 * K];
  __shared__ int sR[8];
  const int s = blockIdx.x;
  const int t = threadIdx.x;
  resolve_taps(s, lv2, lv1, tapsT, sF, sDi);
  const int rs = lv1.rank[s];
  const int na = t < K ? nmi(P - mi[4 * t + 3]) : 0;  // b range of row a = t
  double acc = 0.0;
  for (int i = 0; i < kTapsT; ++i) {
    __syncthreads();
    const int rF = sF[i];
    if (rF < 0) continue;
    if (t < 8) sR[t] = lv0.rank[8 * rF + t];
    const double* Dr = Dil + (size_t)sDi[i] * 8 * K;
    for (int k = t; k < 8 * K; k += NT) sD[k] = Dr[k];
    __syncthreads();
    for (int k = t; k < 8 * K; k += NT) {
      const int o = k / K, b = k - o * K;
      sL[k] = sR[o] >= 0 ? lv0.lbar[(size_t)sR[o] * K + b] : 0.0;
    }
    __syncthreads();
    if (t < K && (rs >= 0 || t == 0)) {
      const int16_t* si = sumidx + (size_t)t * K;
      for (int o = 0; o < 8; ++o) {
        if (sR[o] < 0) continue;
        const double* D = sD + o * K;
        const double* L = sL + o * K;
        for (int b = 0; b < na; ++b) acc += D[si[b]] * L[b];
      }
    }
  }
  if (rs >= 0) {
    if (t < K) lv1.sbar[(size_t)rs * K + t] += acc;
  } else if (t == 0) {
    lv1.mbar[s] += acc;
  }
}

// Source-copy bars -> multipole bars, and M2M^T from the parent (levels
// processed coarse to fine): S_bar[r]_k = c_k 2^|k| Sc_bar[r]_k
//   + sum over the M2M entries (a, k, parity q) of w sign_q(o_r) S_bar[parent]_a.
template <int P>
__global__ __launch_bounds__(256) void k_adj_down(LevelDev lv1, LevelDev lv0, int has_parent, CommonDev cm) {
  constexpr int K = nmi(P);
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= lv0.nref * K) return;
  const int r = i / K, k = i - r * K;
  double v = cm.cfac2[k] * lv0.sbar[i];
  if (has_parent) {
    const int c = lv0.refcell[r];
    const int pr = c >> 3, o = c & 7;
    const double* Sp = lv1.sbar + (size_t)pr * K;
    for (int j = cm.m2mT_start[k]; j < cm.m2mT_start[k + 1]; ++j) {
      const int code = cm.m2mT_list[j];
      v += cm.m2mT_w[j] * parity_sign(code >> 12, o) * Sp[code & 4095];
    }
  }
  lv0.sbar[i] = v;
}

// Mass bars to the caller's slots: leaf cells of rebuilt levels get their own
// bar plus the M2M^T term of their father's multipole bar (monopole entry);
// every other slot of the level gets 0.
template <int P>
__global__ void k_adj_out(LevelDev lv1, LevelDev lv0, int has_parent, int rebuilt, CommonDev cm,
                          double* __restrict__ mbar_out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= lv0.n) return;
  const int s = lv0.slot[c];
  if (s < 0) return;
  double v = 0.0;
  if (rebuilt && lv0.rank[c] < 0) {
    v = lv0.mbar[c];
    if (has_parent) {
      const int o = c & 7;
      const double* Sp = lv1.sbar + (size_t)(c >> 3) * nmi(P);
      for (int j = cm.m2mT_start[0]; j < cm.m2mT_start[1]; ++j) {
        const int code = cm.m2mT_list[j];
        v += cm.m2mT_w[j] * parity_sign(code >> 12, o) * Sp[code & 4095];
      }
    }
  }
  mbar_out[s] = v;
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

hipError_t launch_adj_near(int p, const LevelDev& lv1, const LevelDev& lv0, const LevelDev& lvp, int targets_here,
                           const TablesDev<double>& t64, const CommonDev& cm, hipStream_t st) {
  if (lv1.nref == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_near_leaf, dim3(lv1.nref), dim3(256), 0, st, lv1, lv0, lvp);
  if (!targets_here || !lv0.sbar) return hipGetLastError();
#define X(PP) \
  case PP: hipLaunchKernelGGL((k_adj_near_m2p<PP>), dim3(lv1.nref), dim3(256), 0, st, lv1, lv0, t64.Dsame, t64.cfacn, cm.up); break;
  AFMM_P_SWITCH(p, X)
#undef X
  return hipGetLastError();
}

hipError_t launch_adj_l2p(int p, const LevelDev& lv1, const LevelDev& lv0, const TablesDev<double>& t64,
                          hipStream_t st) {
  if (lv1.nref == 0) return hipSuccess;
#define X(PP) \
  case PP: hipLaunchKernelGGL((k_adj_l2p<PP>), dim3(lv1.nref), dim3(256), 0, st, lv1, lv0, t64.l2p); break;
  AFMM_P_SWITCH(p, X)
#undef X
  return hipGetLastError();
}

hipError_t launch_adj_m2p(int p, const LevelDev& lv2, const LevelDev& lv1, const LevelDev& lv0,
                          const int32_t* tapsT, const TablesDev<double>& t64, const CommonDev& cm, hipStream_t st) {
  if (lv1.n == 0) return hipSuccess;
#define X(PP) \
  case PP: hipLaunchKernelGGL((k_adj_m2p<PP>), dim3(lv1.n), dim3(threads_for(nmi(PP))), 0, st, lv2, lv1, lv0, tapsT, t64.Dil, cm.up); break;
  AFMM_P_SWITCH(p, X)
#undef X
  return hipGetLastError();
}

hipError_t launch_adj_l2l(int p, const LevelDev& lv1, const LevelDev& lv0, const TablesDev<double>& t64,
                          const CommonDev& cm, hipStream_t st) {
  if (lv1.nref == 0) return hipSuccess;
#define X(PP) \
  case PP: hipLaunchKernelGGL((k_adj_l2l<PP>), dim3(lv1.nref), dim3(256), 0, st, lv1, lv0, t64.l2lw, cm.mi); break;
  AFMM_P_SWITCH(p, X)
#undef X
  return hipGetLastError();
}

hipError_t launch_adj_m2l(int p, const LevelDev& lv2, const LevelDev& lv1, const LevelDev& lv0,
                          const int32_t* tapsT, const TablesDev<double>& t64, const CommonDev& cm, hipStream_t st) {
  if (lv1.n == 0) return hipSuccess;
#define X(PP) \
  case PP: hipLaunchKernelGGL((k_adj_m2l<PP>), dim3(lv1.n), dim3(threads_for(nmi(PP))), 0, st, lv2, lv1, lv0, tapsT, t64.Dil, cm.sumidx, cm.mi); break;
  AFMM_P_SWITCH(p, X)
#undef X
  return hipGetLastError();
}

hipError_t launch_adj_down(int p, const LevelDev& lv1, const LevelDev& lv0, int has_parent, const CommonDev& cm,
                           hipStream_t st) {
  const int n = lv0.nref * nmi(p);
  if (n == 0) return hipSuccess;
#define X(PP) \
  case PP: hipLaunchKernelGGL((k_adj_down<PP>), dim3((n + 255) / 256), dim3(256), 0, st, lv1, lv0, has_parent, cm); break;
  AFMM_P_SWITCH(p, X)
#undef X
  return hipGetLastError();
}

hipError_t launch_adj_out(int p, const LevelDev& lv1, const LevelDev& lv0, int has_parent, int rebuilt,
                          const CommonDev& cm, double* mbar_out, hipStream_t st) {
  if (lv0.n == 0) return hipSuccess;
#define X(PP) \
  case PP: hipLaunchKernelGGL((k_adj_out<PP>), dim3((lv0.n + 255) / 256), dim3(256), 0, st, lv1, lv0, has_parent, rebuilt, cm, mbar_out); break;
  AFMM_P_SWITCH(p, X)
#undef X
  return hipGetLastError();
}

#undef AFMM_P_SWITCH

}  // namespace afmm
