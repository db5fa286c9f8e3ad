// HIP kernels of the adaptive FMM for gfx950 (first, VALU form).
//
// Work decomposition.  Targets are grouped by their father F (one "group" =
// the 8 children of one refined cell).  The 8 siblings share one interaction
// list (Sec. 2): the level-(f-1) cells of the 6^3 block around F's oct minus
// the 27 cells touching F, i.e. the children of the 27 neighbours of F's father
// G minus F's own neighbours.  Lists are therefore never stored: each block
// rebuilds its 216 candidates from G's neighbour row and F's octant.
//
// Deterministic: no atomics; every sum runs in a fixed order.
#include <hip/hip_runtime.h>

#include "afmm_internal.h"

namespace afmm {

namespace {

constexpr int kBlock = 256;

inline int ceil_div_host(int a, int b) { return (a + b - 1) / b; }

// Offsets of neighbour e and child octant o along each axis.
__device__ inline int e_axis(int e, int d) { return (d == 0 ? e % 3 : (d == 1 ? (e / 3) % 3 : e / 9)) - 1; }
__device__ inline int o_axis(int o, int d) { return (o >> d) & 1; }
__device__ inline int d_index(int dx, int dy, int dz) { return (dx + 3) + 7 * (dy + 3) + 49 * (dz + 3); }

template <typename T>
__device__ inline T rsqrt_t(T x);
template <>
__device__ inline float rsqrt_t<float>(float x) { return rsqrtf(x); }
template <>
__device__ inline double rsqrt_t<double>(double x) { return 1.0 / sqrt(x); }

// P2P in target-level units: phi~ -= m/|R|, a~ -= m R/|R|^3.
template <typename T>
__device__ inline void p2p(T rx, T ry, T rz, T m, T* out) {
  T r2 = rx * rx + ry * ry + rz * rz;
  T inv = rsqrt_t<T>(r2);
  T w = m * inv;
  T w3 = w * inv * inv;
  out[0] -= w;
  out[1] -= w3 * rx;
  out[2] -= w3 * ry;
  out[3] -= w3 * rz;
}

// M2P of one source multipole with a precomputed D~ row (Taylor series of Sec. 2).
template <typename T, int P>
__device__ inline void m2p(const T* __restrict__ D, const T* __restrict__ S, const T* __restrict__ cf,
                           const int16_t* __restrict__ up, T* out) {
  constexpr int K = nmi(P);
  constexpr int K1 = nmi(P - 1);
  T phi = 0, ax = 0, ay = 0, az = 0;
#pragma unroll 4
  for (int a = 0; a < K1; ++a) {
    T w = cf[a] * S[a];
    phi += w * D[a];
    ax += w * D[up[3 * a + 0]];
    ay += w * D[up[3 * a + 1]];
    az += w * D[up[3 * a + 2]];
  }
#pragma unroll 4
  for (int a = K1; a < K; ++a) phi += cf[a] * S[a] * D[a];
  out[0] += phi;
  out[1] -= ax;
  out[2] -= ay;
  out[3] -= az;
}

// Block-wide compaction of the interaction-list candidates into s_cell/s_d.
// Candidate t (< 216) = child o' = t & 7 of neighbour e = t >> 3 of G; kept if
// inside the box and not touching F.  Returns the count (all threads).
__device__ inline int build_il(const LevelDev& lv2, int G, int oF, int* s_cell, int* s_d, int* s_cnt) {
  const int t = threadIdx.x;
  int cell = -1, di = 0;
  if (t < 216) {
    const int e = t >> 3, op = t & 7;
    const int Q = lv2.nbr[(size_t)G * 27 + e];
    if (Q >= 0) {
      const int rQ = lv2.rank[Q];
      const int dx = 2 * e_axis(e, 0) + o_axis(op, 0) - o_axis(oF, 0);
      const int dy = 2 * e_axis(e, 1) + o_axis(op, 1) - o_axis(oF, 1);
      const int dz = 2 * e_axis(e, 2) + o_axis(op, 2) - o_axis(oF, 2);
      const int dm = max(abs(dx), max(abs(dy), abs(dz)));
      if (dm > 1 && rQ >= 0) {
        cell = 8 * rQ + op;
        di = d_index(dx, dy, dz);
      }
    }
  }
  // wave-level ballot compaction (wave64), then a block prefix over the waves
  const unsigned long long mask = __ballot(cell >= 0);
  const int lane = t & 63, wave = t >> 6;
  const int before = __popcll(mask & ((1ull << lane) - 1ull));
  if (lane == 0) s_cnt[wave] = __popcll(mask);
  __syncthreads();
  int base = 0;
  for (int w = 0; w < wave; ++w) base += s_cnt[w];
  int total = 0;
  for (int w = 0; w < kBlock / 64; ++w) total += s_cnt[w];
  if (cell >= 0) {
    s_cell[base + before] = cell;
    s_d[base + before] = di;
  }
  __syncthreads();
  return total;
}

}  // namespace

// ---------------------------------------------------------------------------
// leaf masses of one level (slot gather); refined cells get 0
__global__ void k_gather_mass(int n, const int32_t* __restrict__ rank, const int32_t* __restrict__ slot,
                              const double* __restrict__ m, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int s = slot[i];
  out[i] = (rank[i] < 0 && s >= 0) ? m[s] : 0.0;
}

hipError_t launch_gather_mass(const LevelDev& lv, const double* m_src, hipStream_t st) {
  if (lv.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_mass, dim3(ceil_div_host(lv.n, 256)), dim3(256), 0, st, lv.n, lv.rank, lv.slot,
                     m_src, lv.mass);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Upward pass (Alg. 2 Upward + CenterShift): P2M of leaf children and M2M of
// refined children into their father's centre, FP64.  One block per father.
template <int P>
__global__ __launch_bounds__(192) void k_upward(LevelDev lv, LevelDev lvc, CommonDev cm, int write32) {
  constexpr int K = nmi(P);
  __shared__ double sc[8 * K];
  const int r = blockIdx.x, t = threadIdx.x;
  for (int i = t; i < 8 * K; i += blockDim.x) {
    const int o = i / K, k = i - o * K;
    const int c = 8 * r + o;
    const int rc = lvc.rank[c];
    sc[i] = rc >= 0 ? lvc.S64[(size_t)rc * K + k] : (k == 0 ? lvc.mass[c] : 0.0);
  }
  __syncthreads();
  if (t < K) {
    double s = 0.0;
    for (int o = 0; o < 8; ++o) {
      const double* row = cm.m2m + ((size_t)o * K + t) * K;
      for (int k = 0; k <= t; ++k) s += row[k] * sc[o * K + k];
    }
    lv.S64[(size_t)r * K + t] = s;
    if (write32) lv.S32[(size_t)r * K + t] = (float)s;
  }
}

// ---------------------------------------------------------------------------
// M2L at FMM level f (Alg. 3): targets are the children y of group F (level
// f-1); sources are F's interaction list at level f-1.  L2L of L[F] is added.
// Thread (o_y = t & 7, j = t >> 3) owns coefficients b = j, j+32, ...
template <typename T, typename TL, int P>
__global__ __launch_bounds__(kBlock) void k_m2l(const int32_t* __restrict__ grp, LevelDev lv2, LevelDev lv1,
                                                LevelDev lv0, TablesDev<T> tb, const TL* __restrict__ Lpar,
                                                const T* __restrict__ Ssrc, T* __restrict__ Lout, CommonDev cm) {
  constexpr int K = nmi(P);
  constexpr int NB = (K + 31) / 32;
  // sources staged per round (LDS budget ~48 KB)
  constexpr int NSRC = (49152 / (9 * K * (int)sizeof(T))) < 8 ? (49152 / (9 * K * (int)sizeof(T))) : 8;
  __shared__ int s_cell[216], s_d[216], s_cnt[4];
  __shared__ T s_S[NSRC][K];              // c_a 2^|a| S~_a
  __shared__ T s_D[NSRC][8][K];           // D~ rows for the 8 child offsets
  const int F = grp[blockIdx.x];
  const int cF = lv1.refcell[F];
  const int t = threadIdx.x;
  const int n = build_il(lv2, cF >> 3, cF & 7, s_cell, s_d, s_cnt);
  const int oy = t & 7, j = t >> 3;
  T acc[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) acc[i] = 0;
  if (Lpar) {
    const TL* LF = Lpar + (size_t)F * K;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int b = j + 32 * i;
      if (b < K) {
        const T* row = tb.l2l + ((size_t)oy * K + b) * K;
        T s = 0;
        for (int k = b; k < K; ++k) s += row[k] * (T)LF[k];
        acc[i] = s;
      }
    }
  }
  for (int s0 = 0; s0 < n; s0 += NSRC) {
    const int ns = min(NSRC, n - s0);
    for (int i = t; i < ns * K; i += kBlock) {
      const int q = i / K, a = i - q * K;
      const int cell = s_cell[s0 + q];
      const int rs = lv1.rank[cell];
      T v;
      if (rs >= 0) v = Ssrc[(size_t)rs * K + a] * tb.cfac2[a];
      else v = a == 0 ? (T)lv1.mass[cell] : (T)0;
      s_S[q][a] = v;
    }
    for (int i = t; i < ns * 8 * K; i += kBlock) {
      const int q = i / (8 * K), rem = i - q * 8 * K;
      const int o = rem / K, g = rem - o * K;
      s_D[q][o][g] = tb.Dil[((size_t)s_d[s0 + q] * 8 + o) * K + g];
    }
    __syncthreads();
    for (int q = 0; q < ns; ++q) {
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int b = j + 32 * i;
        if (b < K) {
          const int16_t* si = cm.sumidx + (size_t)b * K;
          const int na = nmi(P - cm.mi[4 * b + 3]);
          T s = 0;
          for (int a = 0; a < na; ++a) s += s_D[q][oy][si[a]] * s_S[q][a];
          acc[i] += s;
        }
      }
    }
    __syncthreads();
  }
  const int y = 8 * F + oy;
  const int ry = lv0.rank[y];
  if (ry >= 0) {
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int b = j + 32 * i;
      if (b < K) Lout[(size_t)ry * K + b] = acc[i];
    }
  }
}

// ---------------------------------------------------------------------------
// Leaf evaluation at level l (Alg. 4 read through Sec. 3.2): for the leaf
// children of group F, far (L2P of L[F]), intermediate (M2P / P2P over F's
// interaction list at l-1), near (P2P from level-(l-1) and level-l leaves,
// M2P from refined level-l cells not touching the target) and nearest (P2P
// from the children of refined level-l cells touching the target).
// Thread (o = t & 7, j = t >> 3): target child o, every 32nd source from j.
template <typename T, int P>
__global__ __launch_bounds__(kBlock) void k_leaf(const int32_t* __restrict__ grp, int l, LevelDev lv2,
                                                 LevelDev lv1, LevelDev lv0, LevelDev lvp, TablesDev<T> tb,
                                                 const T* __restrict__ Lpar, const T* __restrict__ S1,
                                                 const T* __restrict__ S0, CommonDev cm, double G, double h,
                                                 double* __restrict__ phi, double* __restrict__ acc) {
  constexpr int K = nmi(P);
  __shared__ int s_cell[216], s_d[216], s_cnt[4], s_nb[27];
  __shared__ T s_red[16][kBlock];
  const int F = grp[blockIdx.x];
  const int cF = lv1.refcell[F];
  const int t = threadIdx.x;
  const int o = t & 7, j = t >> 3;
  if (t < 27) s_nb[t] = lv1.nbr[(size_t)F * 27 + t];
  int n = 0;
  if (l >= 2) n = build_il(lv2, cF >> 3, cF & 7, s_cell, s_d, s_cnt);
  else __syncthreads();
  const int cell = 8 * F + o;
  T far[4] = {0, 0, 0, 0}, mid[4] = {0, 0, 0, 0}, nea[4] = {0, 0, 0, 0}, nst[4] = {0, 0, 0, 0};
  const T ox = (T)o_axis(o, 0), oy = (T)o_axis(o, 1), oz = (T)o_axis(o, 2);
  // far field
  if (Lpar) {
    const T* LF = Lpar + (size_t)F * K;
    const T* w = tb.l2p + (size_t)o * 4 * K;
    for (int b = j; b < K; b += 32) {
      const T v = LF[b];
      far[0] += w[b] * v;
      far[1] += w[K + b] * v;
      far[2] += w[2 * K + b] * v;
      far[3] += w[3 * K + b] * v;
    }
  }
  // intermediate field
  for (int k = j; k < n; k += 32) {
    const int s = s_cell[k];
    const int rs = lv1.rank[s];
    const T* D = tb.Dil + ((size_t)s_d[k] * 8 + o) * K;
    if (rs < 0) {
      const T m = (T)lv1.mass[s];
      mid[0] += m * D[0];
      mid[1] -= m * D[1];
      mid[2] -= m * D[2];
      mid[3] -= m * D[3];
    } else {
      m2p<T, P>(D, S1 + (size_t)rs * K, tb.cfac2, cm.up, mid);
    }
  }
  // near and nearest fields
  for (int k = j; k < 216; k += 32) {
    const int e = k >> 3, op = k & 7;
    const int q = s_nb[e];
    if (q < 0) continue;
    const int ex = e_axis(e, 0), ey = e_axis(e, 1), ez = e_axis(e, 2);
    const int rq = lv1.rank[q];
    if (rq < 0) {
      if (op == 0)
        p2p<T>(ox - (T)0.5 - (T)(2 * ex), oy - (T)0.5 - (T)(2 * ey), oz - (T)0.5 - (T)(2 * ez), (T)lv1.mass[q], nea);
      continue;
    }
    const int nc = 8 * rq + op;
    if (nc == cell) continue;
    const int tx = o_axis(o, 0) - 2 * ex - o_axis(op, 0);
    const int ty = o_axis(o, 1) - 2 * ey - o_axis(op, 1);
    const int tz = o_axis(o, 2) - 2 * ez - o_axis(op, 2);
    const int rn = lv0.rank[nc];
    if (rn < 0) {
      p2p<T>((T)tx, (T)ty, (T)tz, (T)lv0.mass[nc], nea);
    } else if (max(abs(tx), max(abs(ty), abs(tz))) <= 1) {
      for (int o2 = 0; o2 < 8; ++o2) {
        const int kc = 8 * rn + o2;
        p2p<T>((T)tx - ((T)o_axis(o2, 0) - (T)0.5) * (T)0.5, (T)ty - ((T)o_axis(o2, 1) - (T)0.5) * (T)0.5,
               (T)tz - ((T)o_axis(o2, 2) - (T)0.5) * (T)0.5, (T)lvp.mass[kc], nst);
      }
    } else {
      const T* D = tb.Dsame + (size_t)d_index(tx, ty, tz) * K;
      m2p<T, P>(D, S0 + (size_t)rn * K, tb.cfac1, cm.up, nea);
    }
  }
  // fixed-order reduction over the 32 threads of each target
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    s_red[c][t] = far[c];
    s_red[4 + c][t] = mid[c];
    s_red[8 + c][t] = nea[c];
    s_red[12 + c][t] = nst[c];
  }
  __syncthreads();
  if (t < 8 && lv0.rank[8 * F + t] < 0) {
    double out[4] = {0, 0, 0, 0};
    for (int c = 0; c < 16; ++c) {
      T s = 0;
      for (int jj = 0; jj < 32; ++jj) s += s_red[c][t + 8 * jj];
      out[c & 3] += (double)s;
    }
    const int sl = lv0.slot[8 * F + t];
    const double sp = G / h, sa = G / (h * h);
    phi[sl] = sp * out[0];
    acc[3 * (size_t)sl + 0] = sa * out[1];
    acc[3 * (size_t)sl + 1] = sa * out[2];
    acc[3 * (size_t)sl + 2] = sa * out[3];
  }
}

// ---------------------------------------------------------------------------
// launchers

hipError_t launch_upward(int p, const LevelDev& lv, const LevelDev& lvc, const CommonDev& cm, bool write32,
                         hipStream_t st) {
  if (lv.nref == 0) return hipSuccess;
  const int K = nmi(p);
  const dim3 grid(lv.nref), block(K <= 64 ? 64 : (K <= 128 ? 128 : 192));
  switch (p) {
#define AFMM_UP(PP) \
  case PP: hipLaunchKernelGGL(k_upward<PP>, grid, block, 0, st, lv, lvc, cm, (int)write32); break;
    AFMM_UP(1) AFMM_UP(2) AFMM_UP(3) AFMM_UP(4) AFMM_UP(5) AFMM_UP(6) AFMM_UP(7) AFMM_UP(8)
#undef AFMM_UP
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, typename TL>
static hipError_t m2l_dispatch(int p, int ngrp, const int32_t* grp, const LevelDev& lv2, const LevelDev& lv1,
                               const LevelDev& lv0, const TablesDev<T>& tb, const TL* Lpar, const T* S, T* Lout,
                               const CommonDev& cm, hipStream_t st) {
  const dim3 grid(ngrp), block(kBlock);
  switch (p) {
#define AFMM_M2L(PP)                                                                                       \
  case PP:                                                                                                 \
    hipLaunchKernelGGL((k_m2l<T, TL, PP>), grid, block, 0, st, grp, lv2, lv1, lv0, tb, Lpar, S, Lout, cm); \
    break;
    AFMM_M2L(1) AFMM_M2L(2) AFMM_M2L(3) AFMM_M2L(4) AFMM_M2L(5) AFMM_M2L(6) AFMM_M2L(7) AFMM_M2L(8)
#undef AFMM_M2L
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_m2l(int p, bool fp32, bool parent_fp32, int f, const int32_t* grp, int ngrp, const LevelDev& lv2,
                      const LevelDev& lv1, const LevelDev& lv0, const TablesDev<float>& t32,
                      const TablesDev<double>& t64, const CommonDev& cm, hipStream_t st) {
  if (ngrp == 0) return hipSuccess;
  const bool has_parent = (f - 1) >= 3;
  if (fp32) {
    if (parent_fp32)
      return m2l_dispatch<float, float>(p, ngrp, grp, lv2, lv1, lv0, t32, has_parent ? lv1.L32 : nullptr, lv1.S32,
                                        lv0.L32, cm, st);
    return m2l_dispatch<float, double>(p, ngrp, grp, lv2, lv1, lv0, t32, has_parent ? lv1.L64 : nullptr, lv1.S32,
                                       lv0.L32, cm, st);
  }
  return m2l_dispatch<double, double>(p, ngrp, grp, lv2, lv1, lv0, t64, has_parent ? lv1.L64 : nullptr, lv1.S64,
                                      lv0.L64, cm, st);
}

template <typename T>
static hipError_t leaf_dispatch(int p, int l, int ngrp, const int32_t* grp, const LevelDev& lv2, const LevelDev& lv1,
                                const LevelDev& lv0, const LevelDev& lvp, const TablesDev<T>& tb, const T* Lpar,
                                const T* S1, const T* S0, const CommonDev& cm, double G, double h, double* phi,
                                double* acc, hipStream_t st) {
  const dim3 grid(ngrp), block(kBlock);
  switch (p) {
#define AFMM_LEAF(PP)                                                                                          \
  case PP:                                                                                                     \
    hipLaunchKernelGGL((k_leaf<T, PP>), grid, block, 0, st, grp, l, lv2, lv1, lv0, lvp, tb, Lpar, S1, S0, cm, G, \
                       h, phi, acc);                                                                           \
    break;
    AFMM_LEAF(1) AFMM_LEAF(2) AFMM_LEAF(3) AFMM_LEAF(4) AFMM_LEAF(5) AFMM_LEAF(6) AFMM_LEAF(7) AFMM_LEAF(8)
#undef AFMM_LEAF
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_leaf(int p, bool fp32, int l, const int32_t* grp, int ngrp, const LevelDev& lv2,
                       const LevelDev& lv1, const LevelDev& lv0, const LevelDev& lvp,
                       const TablesDev<float>& t32, const TablesDev<double>& t64, const CommonDev& cm, double G,
                       double h, double* phi, double* acc, hipStream_t st) {
  if (ngrp == 0) return hipSuccess;
  const bool has_far = (l - 1) >= 3;
  if (fp32)
    return leaf_dispatch<float>(p, l, ngrp, grp, lv2, lv1, lv0, lvp, t32, has_far ? lv1.L32 : nullptr, lv1.S32,
                                lv0.S32, cm, G, h, phi, acc, st);
  return leaf_dispatch<double>(p, l, ngrp, grp, lv2, lv1, lv0, lvp, t64, has_far ? lv1.L64 : nullptr, lv1.S64,
                               lv0.S64, cm, G, h, phi, acc, st);
}

}  // namespace afmm
