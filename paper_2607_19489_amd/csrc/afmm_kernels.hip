// HIP kernels of the adaptive FMM for gfx950.
//
// Group = the 8 children of one refined cell F.  The 8 siblings share F's
// interaction list (Sec. 2): the level-(f-1) cells of the 6^3 block around
// F's oct minus the 27 cells touching F, i.e. the children of the 27
// neighbours of F's father G minus F's own neighbours.  Relative to F the
// source offsets d = s - F form a fixed set of 189 "taps" that depends only on
// F's octant (parity class), and the translation operator of a tap depends
// only on d and the child octant.  Groups of one parity class therefore share
// every operator: M2L and the intermediate-field M2P become, tap by tap, dense
// products  OUT[rows x groups] += A_d[rows x K] * S[K x groups]  on MFMA.
//
// Deterministic: no atomics; every sum runs in a fixed order.
#include <hip/hip_runtime.h>
#include <algorithm>

#include "afmm_internal.h"
#include "afmm_mfma.h"

namespace afmm {

namespace {

constexpr int kBlock = 256;
constexpr int kTaps = 189;

inline int ceil_div_host(int a, int b) { return (a + b - 1) / b; }

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
  const T r2 = rx * rx + ry * ry + rz * rz;
  const T inv = rsqrt_t<T>(r2);
  const T w = m * inv;
  const T w3 = w * inv * inv;
  out[0] -= w;
  out[1] -= w3 * rx;
  out[2] -= w3 * ry;
  out[3] -= w3 * rz;
}

// Compile-time multi-index tables of order P: degree |a| and the position of
// a + e_i (or -1 when |a| = P) for every degree-ordered position a.
template <int P>
struct MiTab {
  int deg[nmi(P)];
  int up[nmi(P)][3];
  constexpr MiTab() : deg(), up() {
    for (int n = 0; n <= P; ++n)
      for (int a = n; a >= 0; --a)
        for (int b = n - a; b >= 0; --b) {
          const int c = n - a - b, g = mi_index(a, b, c);
          deg[g] = n;
          for (int i = 0; i < 3; ++i)
            up[g][i] = n < P ? mi_index(a + (i == 0), b + (i == 1), c + (i == 2)) : -1;
        }
  }
};

// M2P of one multipole with a D~ row, for the near field (VALU): fully
// unrolled over the coefficients, so every D~ and source index (and the
// weight 2^-|a| of the same-level source copy) is a compile-time constant.
template <typename T, int P>
__device__ inline void m2p_row(const T* __restrict__ D, const T* __restrict__ S, T* out) {
  constexpr int K = nmi(P);
  constexpr int K1 = nmi(P - 1);
  constexpr MiTab<P> mt{};
  T phi = 0, ax = 0, ay = 0, az = 0;
#pragma unroll
  for (int a = 0; a < K1; ++a) {
    const T w = (T)(1.0 / (double)(1 << mt.deg[a])) * S[src_pos(a, (int)sizeof(T))];
    phi += w * D[a];
    ax += w * D[mt.up[a][0]];
    ay += w * D[mt.up[a][1]];
    az += w * D[mt.up[a][2]];
  }
#pragma unroll
  for (int a = K1; a < K; ++a) phi += (T)(1.0 / (double)(1 << mt.deg[a])) * S[src_pos(a, (int)sizeof(T))] * D[a];
  out[0] += phi;
  out[1] -= ax;
  out[2] -= ay;
  out[3] -= az;
}

}  // namespace

// ---------------------------------------------------------------------------
// leaf masses of one level (slot gather); refined cells get 0
__global__ void k_gather_mass(int n, const int32_t* __restrict__ rank, const int32_t* __restrict__ slot,
                              const double* __restrict__ m, double* __restrict__ out, double* __restrict__ snap) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int s = slot[i];
  const double v = s >= 0 ? m[s] : 0.0;
  out[i] = rank[i] < 0 ? v : 0.0;
  if (snap && s >= 0) snap[s] = v;
}

hipError_t launch_gather_mass(const LevelDev& lv, const double* m_src, double* snap, hipStream_t st) {
  if (lv.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_mass, dim3(ceil_div_host(lv.n, 256)), dim3(256), 0, st, lv.n, lv.rank, lv.slot,
                     m_src, lv.mass, snap);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Upward pass (Alg. 2 Upward + CenterShift), FP64.  With child offsets
// d_o = (o - 1/2)/2 the M2M weight C(a,k) d_o^(a-k) 2^-|k| splits into
// C(a,k) 4^-|a-k| 2^-|k| times a sign that depends only on the parity of
// a - k, so the 8 children are first folded into 8 signed sums per
// coefficient:  Y[k][q] = sum_o (prod_{i: q_i=1} sgn(o_i)) S_o[k].
// The weights C(a,k) 4^-|a-k| 2^-|k| and signs are tabulated per coefficient a
// (cm.m2m_list: for each a, its (k, parity) entries; cm.m2m_w the weights).
// Thread = (cell, coefficient) over chunks of CB cells; a block is persistent:
// it stages the entry tables in LDS once, then for each chunk loads the
// children's ranks and masses, forms the 8 signed child sums Y of each cell in
// LDS and sums the entries of each coefficient.
// The source copies are written in the lane-group layout; thread a >= K of a
// cell writes the zero of padding slot src_pos(a).  Runs over a list of the
// level's refined ranks (those with a refined child; k_p2m_leaf takes the
// others).
template <int P>
__global__ __launch_bounds__(256) void k_upward(const int32_t* __restrict__ list, int nlist, LevelDev lv,
                                                LevelDev lvc, CommonDev cm) {
  constexpr int K = nmi(P);
  constexpr int NE = nmi_entries(P);
  constexpr int STP32 = src_stp(P, 4), STP64 = src_stp(P, 8);
  constexpr int KP = 4 * STP32;               // threads per cell (STP32 >= STP64)
  constexpr int CB = 256 / KP;                // cells per chunk
  __shared__ double sY[CB][8][K];
  __shared__ double sW[NE];
  __shared__ int sE[NE];
  __shared__ int sB[K + 1];
  __shared__ int sRc[CB][8];
  __shared__ double sM[CB][8];
  const int t = threadIdx.x;
  for (int i = t; i < NE; i += 256) {
    sW[i] = cm.m2m_w[i];
    sE[i] = cm.m2m_list[i];
  }
  for (int i = t; i <= K; i += 256) sB[i] = cm.m2m_start[i];
  const int c = t / KP, a = t - c * KP;
  // children of a chunk: refined rank and mass (the gathered mass of a refined
  // child is 0 and unused), two independent loads, prefetched one chunk ahead
  auto child = [&](int i0, int& rc, double& m) {
    rc = -1;
    m = 0.0;
    const int i = i0 + (t >> 3);
    if (t < CB * 8 && i < nlist) {
      const int ch = 8 * list[i] + (t & 7);
      rc = lvc.rank[ch];
      m = lvc.mass[ch];
    }
  };
  int rcn;
  double mn;
  child(blockIdx.x * CB, rcn, mn);
  for (int i0 = blockIdx.x * CB; i0 < nlist; i0 += gridDim.x * CB) {
    if (t < CB * 8) {
      sRc[t >> 3][t & 7] = rcn;
      sM[t >> 3][t & 7] = rcn < 0 ? mn : 0.0;
    }
    child(i0 + gridDim.x * CB, rcn, mn);
    __syncthreads();
    // a cell whose 8 children are leaves has only monopole children: its signed
    // sums vanish for k > 0 and each coefficient keeps the k = 0 entry (the
    // first of its list)
    auto leaf_only = [&](int cc) {
      bool lo = true;
#pragma unroll
      for (int o = 0; o < 8; ++o) lo = lo && sRc[cc][o] < 0;
      return lo;
    };
    // 8 child values per (cell, coefficient) -> signed sums over the octant bits
    for (int i = t; i < CB * K; i += 256) {
      const int cc = i / K, k = i - cc * K;
      if (k > 0 && leaf_only(cc)) continue;
      double v[8];
#pragma unroll
      for (int o = 0; o < 8; ++o) {
        const int rc = sRc[cc][o];
        v[o] = rc >= 0 ? lvc.S64[(size_t)rc * K + k] : (k == 0 ? sM[cc][o] : 0.0);
      }
#pragma unroll
      for (int bit = 0; bit < 3; ++bit) {
        double u[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int qlo = q & ~(1 << bit);
          u[q] = (q & (1 << bit)) ? v[qlo | (1 << bit)] - v[qlo] : v[qlo] + v[qlo | (1 << bit)];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = u[q];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) sY[cc][q][k] = v[q];
    }
    __syncthreads();
    const int r = i0 + c < nlist ? list[i0 + c] : -1;
    if (c < CB && r >= 0) {
      if (a >= K) {  // zero padding of the source copies
        if (lv.S32) lv.S32[(size_t)r * 4 * STP32 + src_pos(a, 4)] = 0.f;
        if (lv.Sc64 && a < 4 * STP64) lv.Sc64[(size_t)r * 4 * STP64 + src_pos(a, 8)] = 0.0;
      } else {
        double acc = 0.0;
        if (leaf_only(c)) {
          acc = sW[sB[a]] * sY[c][sE[sB[a]] >> 12][0];
        } else {
          for (int j = sB[a]; j < sB[a + 1]; ++j) {
            const int e = sE[j];
            acc += sW[j] * sY[c][e >> 12][e & 4095];
          }
        }
        lv.S64[(size_t)r * K + a] = acc;
        // source copies for the translation kernels carry the factor (-1)^|a|/a! 2^|a|
        const double sc = acc * cm.cfac2[a];
        if (lv.S32) lv.S32[(size_t)r * 4 * STP32 + src_pos(a, 4)] = (float)sc;
        if (lv.Sc64) lv.Sc64[(size_t)r * 4 * STP64 + src_pos(a, 8)] = sc;
      }
    }
    __syncthreads();
  }
}

// Upward pass for the refined cells whose 8 children are leaves (P2M, Eq.
// eq:P2M): the signed child sums vanish for k > 0, so coefficient a is the
// k = 0 entry of its M2M list times one signed sum of the 8 masses (signs by
// the parity of a).  A block takes kP2mCells cells of the list: their masses
// go to LDS, thread (cell, a) forms coefficient a once, and the three copies
// (S64 in coefficient order, the scaled FP32 and FP64 copies in their
// lane-group layouts) are written slot by slot in row order, so consecutive
// threads store consecutive addresses (padding slots get 0).
constexpr int kP2mCells = 8;

template <int P>
__global__ __launch_bounds__(256) void k_p2m_leaf(const int32_t* __restrict__ list, int nlist, LevelDev lv,
                                                  LevelDev lvc, CommonDev cm) {
  constexpr int K = nmi(P);
  constexpr int R32 = src_row(P, 4), R64 = src_row(P, 8);
  constexpr int NC = kP2mCells;
  __shared__ int sR[NC];
  __shared__ double sM[NC][8];
  __shared__ double sV[NC][K];
  const int t = threadIdx.x;
  const int c0 = blockIdx.x * NC;
  const int nc = min(NC, nlist - c0);
  if (t < NC) sR[t] = t < nc ? list[c0 + t] : -1;
  __syncthreads();
  if (t < 8 * nc) sM[t >> 3][t & 7] = as_global(lvc.mass)[8 * (size_t)sR[t >> 3] + (t & 7)];
  __syncthreads();
  for (int i = t; i < nc * K; i += 256) {
    const int c = i / K, a = i - c * K;
    double v[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) v[o] = sM[c][o];
    const int e0 = cm.m2m_start[a];
    const int q = cm.m2m_list[e0] >> 12;
    // signed sum over the octant bits of q (the butterfly of k_upward, one output)
#pragma unroll
    for (int bit = 0; bit < 3; ++bit) {
      double u[8];
#pragma unroll
      for (int o = 0; o < 8; ++o) {
        const int lo = o & ~(1 << bit);
        u[o] = (q & (1 << bit)) ? v[lo | (1 << bit)] - v[lo] : v[lo] + v[lo | (1 << bit)];
      }
#pragma unroll
      for (int o = 0; o < 8; ++o) v[o] = u[o];
    }
    sV[c][a] = cm.m2m_w[e0] * v[q];
  }
  __syncthreads();
  // coefficient of slot s of a lane-group-layout row (inverse of src_pos), or
  // K for a padding slot
  auto slot_coef = [](int s, int vw) {
    const int j = s / (4 * vw), g = (s % (4 * vw)) / vw, e = s % vw;
    const int k = 4 * (vw * j + e) + g;
    return k < K ? k : K;
  };
  for (int i = t; i < nc * K; i += 256) {
    const int c = i / K, a = i - c * K;
    lv.S64[(size_t)sR[c] * K + a] = sV[c][a];
  }
  if (lv.S32)
    for (int i = t; i < nc * R32; i += 256) {
      const int c = i / R32, sl = i - c * R32, k = slot_coef(sl, 4);
      lv.S32[(size_t)sR[c] * R32 + sl] = k < K ? (float)(sV[c][k] * cm.cfac2[k]) : 0.f;
    }
  if (lv.Sc64)
    for (int i = t; i < nc * R64; i += 256) {
      const int c = i / R64, sl = i - c * R64, k = slot_coef(sl, 2);
      lv.Sc64[(size_t)sR[c] * R64 + sl] = k < K ? sV[c][k] * cm.cfac2[k] : 0.0;
    }
}

__global__ void k_batch_in(int64_t nleaf, const int32_t* __restrict__ leafslot, const int32_t* __restrict__ leafhier,
                           const int64_t* __restrict__ base, const double* const* __restrict__ mass,
                           double* __restrict__ m_forest) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nleaf) return;
  const int32_t s = leafslot[i], h = leafhier[i];
  m_forest[s] = mass[h][s - base[h]];
}

__global__ void k_batch_out(int64_t nleaf, const int32_t* __restrict__ leafslot, const int32_t* __restrict__ leafhier,
                            const int64_t* __restrict__ base, const double* __restrict__ phi_forest,
                            const double* __restrict__ acc_forest, double* const* __restrict__ phi,
                            double* const* __restrict__ acc) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nleaf) return;
  const int32_t s = leafslot[i], h = leafhier[i];
  const int64_t j = s - base[h];
  phi[h][j] = phi_forest[s];
  acc[h][3 * j + 0] = acc_forest[3 * (int64_t)s + 0];
  acc[h][3 * j + 1] = acc_forest[3 * (int64_t)s + 1];
  acc[h][3 * j + 2] = acc_forest[3 * (int64_t)s + 2];
}

hipError_t launch_batch_in(int64_t nleaf, const int32_t* leafslot, const int32_t* leafhier, const int64_t* base,
                           const double* const* mass, double* m_forest, hipStream_t st) {
  if (nleaf <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_in, dim3((unsigned)((nleaf + 255) / 256)), dim3(256), 0, st, nleaf, leafslot, leafhier,
                     base, mass, m_forest);
  return hipGetLastError();
}

hipError_t launch_batch_out(int64_t nleaf, const int32_t* leafslot, const int32_t* leafhier, const int64_t* base,
                            const double* phi_forest, const double* acc_forest, double* const* phi,
                            double* const* acc, hipStream_t st) {
  if (nleaf <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_out, dim3((unsigned)((nleaf + 255) / 256)), dim3(256), 0, st, nleaf, leafslot,
                     leafhier, base, phi_forest, acc_forest, phi, acc);
  return hipGetLastError();
}

hipError_t launch_upward(int p, const int32_t* leaf, int nleaf, const int32_t* mix, int nmix, const LevelDev& lv,
                         const LevelDev& lvc, const CommonDev& cm, hipStream_t st) {
  const int KP = src_row(p, 4), CB = 256 / KP;
  if (nleaf > 0) {
    const dim3 grid((unsigned)((nleaf + kP2mCells - 1) / kP2mCells)), block(256);
    switch (p) {
#define AFMM_P2M(PP) \
  case PP: hipLaunchKernelGGL(k_p2m_leaf<PP>, grid, block, 0, st, leaf, nleaf, lv, lvc, cm); break;
      AFMM_P2M(1) AFMM_P2M(2) AFMM_P2M(3) AFMM_P2M(4) AFMM_P2M(5) AFMM_P2M(6) AFMM_P2M(7) AFMM_P2M(8)
#undef AFMM_P2M
      default: return hipErrorInvalidValue;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (nmix > 0) {
    // persistent blocks: a few per CU, each looping over chunks of CB cells
    const dim3 grid(std::min((nmix + CB - 1) / CB, 8 * 256)), block(kBlock);
    switch (p) {
#define AFMM_UP(PP) \
  case PP: hipLaunchKernelGGL(k_upward<PP>, grid, block, 0, st, mix, nmix, lv, lvc, cm); break;
      AFMM_UP(1) AFMM_UP(2) AFMM_UP(3) AFMM_UP(4) AFMM_UP(5) AFMM_UP(6) AFMM_UP(7) AFMM_UP(8)
#undef AFMM_UP
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Completion of the local expansions of FMM level f (one block per M2L group
// F): L~_b[y] = sum_c Lpart[c][y]_b (the M2L tap sums, split over `nsplit`
// tap ranges, added in fixed order; or the single sum already in L) + the
// ShiftLocal term sum_g w_o[|b|][g] L~_{b+g}[F] (Eq. eq:L2L) when F has one.
// Three passes over the group's 8K coefficients through LDS: the tap sums
// and the stores run coefficient-fastest (whole child rows per wave), the
// shift sums child-fastest; the sums and their order are unchanged.  NS
// bounds the split (1: the single sum in L): every partial of every
// coefficient a thread owns is loaded at once, so a block waits for one
// round of loads rather than one per four partials and coefficient.
template <typename T, typename TL, int P, int NS>
__global__ __launch_bounds__(kBlock) void k_l2l(const int32_t* __restrict__ grp, const TL* __restrict__ Lpar,
                                                const int32_t* __restrict__ rank0, T* __restrict__ Lout,
                                                const T* __restrict__ Lpart, int nsplit, size_t split_stride,
                                                const T* __restrict__ w, const int16_t* __restrict__ sumidx,
                                                const int8_t* __restrict__ mi) {
  constexpr int K = nmi(P);
  constexpr int KV = K | 1;  // odd LDS row stride: the 8 rows of a wave's loads fall in different banks
  __shared__ T sL[K];
  __shared__ T sV[8 * KV];
  __shared__ int sRy[8];
  const int F = grp[blockIdx.x];
  const int t = threadIdx.x;
  if (t < K && Lpar) sL[t] = (T)Lpar[(size_t)F * K + t];
  if (t < 8) sRy[t] = rank0[8 * F + t];
  __syncthreads();
  // tap sums, coefficient fastest (each child's row is read contiguously);
  // a thread owns coefficients t, t + 256, ... (NI of them); a missing child
  // row reads row 0 and is not stored
  constexpr int NI = (8 * K + kBlock - 1) / kBlock;
  {
    T x[NI][NS];
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int i = min(t + kBlock * j, 8 * K - 1), o = i / K, b = i - o * K;
      const int ry = sRy[o];
      const size_t at = (size_t)(ry >= 0 ? ry : 0) * K + b;
#pragma unroll
      for (int c = 0; c < NS; ++c) x[j][c] = NS == 1 ? Lout[at] : Lpart[min(c, nsplit - 1) * split_stride + at];
    }
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int i = t + kBlock * j;
      if (i >= 8 * K) break;
      const int o = i / K, b = i - o * K;
      if (sRy[o] < 0) continue;
      T v = 0;
      if constexpr (NS == 1) {
        v = x[j][0];
      } else {
#pragma unroll
        for (int c = 0; c < NS; ++c)
          if (c < nsplit) v += x[j][c];
      }
      sV[o * KV + b] = v;
    }
  }
  __syncthreads();
  // ShiftLocal, child o fastest: the lanes of a wave share few coefficients
  // b, all of nearly the same degree, so their shift sums have nearly equal
  // lengths
  if (Lpar) {
    for (int i = t; i < 8 * K; i += kBlock) {
      const int o = i & 7, b = i >> 3;
      if (sRy[o] < 0) continue;
      const int nb = mi[4 * b + 3];
      const T* wr = w + ((size_t)o * (P + 1) + nb) * K;
      const int16_t* si = sumidx + (size_t)b * K;
      T sh = 0;
      for (int g = 0; g < nmi(P - nb); ++g) sh += wr[g] * sL[si[g]];
      sV[o * KV + b] += sh;
    }
    __syncthreads();
  }
  for (int i = t; i < 8 * K; i += kBlock) {
    const int o = i / K, b = i - o * K;
    const int ry = sRy[o];
    if (ry >= 0) Lout[(size_t)ry * K + b] = sV[o * KV + b];
  }
}

// ---------------------------------------------------------------------------
// Shared tap pipeline of the MFMA kernels.  A block owns 16 groups of one
// parity class at one level.  For each of the 189 taps:
//   B[k][n] = c_k 2^|k| S~_k of the tap's source of group n (monopole for a
//             leaf source, 0 when there is none) is loaded by lane (n, g)
//             straight into registers: its STP coefficients k = 4 kb + g are
//             runs of the source copy (lane-group layout: 16-byte vector j of
//             the 4 lane groups adjacent, so a load reads 64 B of each row);
//   sD[o][g] = D~_g at the tap's child offset o (8 rows, then one zero slot)
//             is staged in LDS while the MFMAs of the previous tap run.
// A fragments are read from sD through per-lane offsets that do not depend on
// the tap (kept in registers).
template <typename T, int P>
struct TapStage {
  static constexpr int K = nmi(P);
  static constexpr int KP = (K + 3) & ~3;    // coefficients covered by the k-steps
  static constexpr int KS = dstage_ks(P);    // sD row stride
  static constexpr int VW = 16 / (int)sizeof(T);
  static constexpr int STP = src_stp(P, (int)sizeof(T));  // per-lane run of the source copy
  static constexpr int ROW = 4 * STP;        // source-copy row length
  static constexpr int NVB = STP / VW;       // 16-byte vectors per lane and tap
  static constexpr int SD = 8 * KS + 1;      // sD size (8 rows + zero slot)
  static constexpr int SDP = dstage_len(P, (int)sizeof(T));  // staged length (16-byte padded)
  static constexpr int NDV = SDP / VW;       // 16-byte vectors of one stage
  static_assert(KS == dstage_ks(P), "stage stride");
};

// scaled source copies c_a 2^|a| S~_a of a level
template <typename T> __device__ inline const T* level_S(const LevelDev& lv);
template <> __device__ inline const float* level_S<float>(const LevelDev& lv) { return lv.S32; }
template <> __device__ inline const double* level_S<double>(const LevelDev& lv) { return lv.Sc64; }
template <typename T> __device__ inline T* level_L(const LevelDev& lv);
template <> __device__ inline float* level_L<float>(const LevelDev& lv) { return lv.L32; }
template <> __device__ inline double* level_L<double>(const LevelDev& lv) { return lv.L64; }

// Drops the taps of a range that have no source in any of the 16 columns
// (they add nothing; common near the box faces), keeping the order: run by
// one whole wave, in place on the source table src[tap][16], with the taps'
// codes copied to code[].  Returns the number kept (at least 1: an empty
// range keeps its first tap, whose B is zero).
__device__ inline int compact_taps(int nt, const int32_t* __restrict__ tp, int* src, int* code) {
  const int lane = threadIdx.x & 63;
  int cnt = 0;
  for (int i0 = 0; i0 < nt; i0 += 64) {
    const int i = i0 + lane;
    int v[16];
    bool any = false;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      v[c] = i < nt ? src[i * 16 + c] : -1;
      any = any || v[c] != -1;
    }
    const int cd = i < nt ? tp[i] : 0;
    const uint64_t m = __ballot(any);
    wave_sync();
    if (any) {
      const int j = cnt + __popcll(m & ((1ull << lane) - 1ull));
#pragma unroll
      for (int c = 0; c < 16; ++c) src[j * 16 + c] = v[c];
      code[j] = cd;
    }
    cnt += __popcll(m);
    wave_sync();
  }
  if (cnt == 0) {
    if (lane < 16) src[lane] = -1;
    if (lane == 0) code[0] = tp[0];
    cnt = 1;
  }
  wave_sync();
  return cnt;
}

// Tap range of chunk c of nsplit: whole pairs of taps (the tap loops run in
// pairs), so that only the last chunk has an odd count and runs one empty tap.
// The host keeps nsplit <= 21, so every range holds at least 8 taps.
__host__ __device__ inline void tap_range(int c, int nsplit, int& tb, int& te) {
  constexpr int kPairs = (kTaps + 1) / 2;
  tb = 2 * (c * kPairs / nsplit);
  te = min(kTaps, 2 * ((c + 1) * kPairs / nsplit));
}

// Source of column n for tap `code`: refined rank (>= 0), -2 - cell for a leaf
// (monopole), or -1 when there is none.  The tap loops resolve the sources of
// all their taps into LDS before the loop.
__device__ inline int tap_src(int code, int n, const int* __restrict__ sCB, gptr<int32_t> rank1) {
  const int cb = sCB[n * 27 + (code & 31)];
  const int s = cb < 0 ? -1 : cb + ((code >> 5) & 7);
  if (s < 0) return -1;
  const int rs = rank1[s];
  return rs >= 0 ? rs : -2 - s;
}

// B fragments of one tap for lane (n = lane & 15, g = lane >> 4): the lane's
// run of steps (16-byte vector j holds steps VW j .. VW j + VW - 1), without a
// branch: a missing or leaf source reads the zero row zrow after the level's
// nref rows, and every lane loads a mass (cell 0 when the source is no leaf),
// put into the monopole slot when the tap is used (bfrag_m0).  Only the NS
// steps used are loaded (a partial last vector element by element): an
// element loaded but never read would leave a register that the compiler
// reuses while the load is still in flight.
template <typename T, int P, int NS>
__device__ inline void load_bfrag_nb(int sr, int zrow, gptr<double> mass1, gptr<T> S1,
                                     typename Vec16<T>::type* vb, double& vm) {
  using TS = TapStage<T, P>;
  using V = typename Vec16<T>::type;
  constexpr int NF = NS / TS::VW, R = NS % TS::VW;
  gptr<T> src = S1 + (size_t)(sr >= 0 ? sr : zrow) * TS::ROW;
  const int g = (threadIdx.x & 63) >> 4;
#pragma unroll
  for (int j = 0; j < NF; ++j) vb[j] = *(gptr<V>)(src + src_vec(j, g, (int)sizeof(T)));
#pragma unroll
  for (int r = 0; r < R; ++r) vb[NF][r] = src[src_vec(NF, g, (int)sizeof(T)) + r];
  vm = mass1[sr <= -2 ? -2 - sr : 0];
}
template <typename T>
__device__ inline T bfrag_m0(int sr, double vm, T b0) {
  return (sr <= -2 && ((threadIdx.x & 63) >> 4) == 0) ? (T)vm : b0;
}

// The same run of steps loaded row by row: lane 4 r + q takes vector j of lane
// group q of row r, so the 4 lanes of every quad read one contiguous 64-byte
// piece of one row (one cache-line lookup per quad instead of four), and step
// kb of column n, group g is then found in lane 4 n + g (xb_take).
template <typename T, int P, int NS>
__device__ inline void load_brows_xb(int rr, int zrow, gptr<T> S1, typename Vec16<T>::type* vb) {
  using TS = TapStage<T, P>;
  using V = typename Vec16<T>::type;
  constexpr int NF = NS / TS::VW, R = NS % TS::VW;
  gptr<T> src = S1 + (size_t)(rr >= 0 ? rr : zrow) * TS::ROW;
  const int q = threadIdx.x & 3;
#pragma unroll
  for (int j = 0; j < NF; ++j) vb[j] = *(gptr<V>)(src + src_vec(j, q, (int)sizeof(T)));
#pragma unroll
  for (int r = 0; r < R; ++r) vb[NF][r] = src[src_vec(NF, q, (int)sizeof(T)) + r];
}
// B fragment value of this lane from the lane whose byte address is xa (the
// cross-lane crossbar; no LDS memory is touched)
__device__ inline float xb_take(int xa, float v) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(xa, __float_as_int(v)));
}
__device__ inline double xb_take(int xa, double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(xa, (int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_ds_bpermute(xa, (int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// D~ stage of tap `code` (rows already in the LDS layout): NTH threads copy
// its NDV 16-byte vectors, thread t taking vectors t, t + NTH, ...
template <typename T, int P, int NTH>
__device__ inline void load_dstage(int code, const T* __restrict__ Dst, typename Vec16<T>::type* vD) {
  using TS = TapStage<T, P>;
  using V = typename Vec16<T>::type;
  constexpr int NJ = (TS::NDV + NTH - 1) / NTH;
  const int t = threadIdx.x;
  const V* src = (const V*)(Dst + (size_t)(code >> 8) * TS::SDP);
#pragma unroll
  for (int j = 0; j < NJ; ++j)
    if (TS::NDV % NTH == 0 || t + NTH * j < TS::NDV) vD[j] = src[t + NTH * j];
}

template <typename T, int P, int NTH>
__device__ inline void store_dstage(T* sD, const typename Vec16<T>::type* vD) {
  using TS = TapStage<T, P>;
  using V = typename Vec16<T>::type;
  constexpr int NJ = (TS::NDV + NTH - 1) / NTH;
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < NJ; ++j)
    if (TS::NDV % NTH == 0 || t + NTH * j < TS::NDV) ((V*)sD)[t + NTH * j] = vD[j];
}

// Block-local setup: the tile record (level, then NC groups) and, per group,
// the child base (8 x refined rank) of each of its father's 27 neighbours.
__device__ inline void tile_setup(const int32_t* __restrict__ rec, int NC, const LevelDev& lv2,
                                  const LevelDev& lv1, int* sF, int* sCB) {
  const int t = threadIdx.x;
  if (t < NC) sF[t] = rec[1 + t];
  __syncthreads();
  for (int i = t; i < NC * 27; i += kBlock) {
    const int n = i / 27, e = i - n * 27;
    const int F = sF[n];
    int v = -1;
    if (F >= 0) {
      const int G = as_global(lv1.refcell)[F] >> 3;
      const int Q = as_global(lv2.nbr)[(size_t)G * 27 + e];
      if (Q >= 0) {
        const int rQ = as_global(lv2.rank)[Q];
        if (rQ >= 0) v = 8 * rQ;
      }
    }
    sCB[i] = v;
  }
}


// ---------------------------------------------------------------------------
// Intermediate-field M2P at the leaves (Alg. 4 / Sec. 3.2): rows = 8 children
// x (phi, ax, ay, az) in two 16-row tiles (the acceleration rows only need
// multipoles of order < p), columns = 16 groups of one parity class,
// K = multipole coefficients.  One wave per block: B comes straight from the
// source copies into registers (the next tap's while the current tap's MFMAs
// run), only the D~ rows go through LDS.  Output: part[F][c*8+o]
// (accelerations already negated), in target-level units.  One launch covers
// the tiles of every level of one precision.  One block takes one of `nsplit`
// contiguous tap ranges of its tile and writes its own partial set
// part[chunk][F][...], summed in order by the leaf kernel.
// For FP32 from p = 6 on the launcher sizes the LDS source table for 2 waves
// per SIMD (the best measured there); the same bound lets the compiler use the
// registers of that occupancy.
// XB (tile shape 3): the B rows are loaded row by row (load_brows_xb) and each
// step's fragment is taken from its lane over the crossbar, which cuts the L1
// tag lookups of the B loads by 4x; the MFMAs, operands and order are those of
// the direct form, so the results are identical.
template <typename T, int P, bool XB>
constexpr int m2p_max_waves() { return sizeof(T) == 4 && P >= 6 ? (XB ? 4 : 2) : 8; }

template <typename T, int P, bool XB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(XB && sizeof(T) == 4 && P == 6 ? 4 : 1, m2p_max_waves<T, P, XB>()))) void k_m2p(const int32_t* __restrict__ tiles, int ntiles, int nsplit,
                                            const int32_t* __restrict__ taps, const int16_t* __restrict__ aoff,
                                            const LevelDev* __restrict__ lvs, const T* __restrict__ Dst) {
  using TS = TapStage<T, P>;
  using V = typename Vec16<T>::type;
  constexpr int K1 = nmi(P - 1);
  constexpr int ST0 = TS::KP / 4, ST1 = ((K1 + 3) & ~3) / 4;
  constexpr int NV = (ST0 + TS::VW - 1) / TS::VW;
  constexpr int ND = (TS::NDV + 63) / 64;
  __shared__ __align__(16) T sD[2][TS::SDP];
  __shared__ int sF[16];
  __shared__ int sCB[16 * 27];
  extern __shared__ int sSrcT[];  // [taps of the longest range][16], sized by the launcher
  const int item = xcd_tile(ntiles * nsplit);
  if (item >= ntiles * nsplit) return;
  const int tile = item / nsplit, chunk = item - tile * nsplit;
  int tb, te;
  tap_range(chunk, nsplit, tb, te);
  const int lane = threadIdx.x;
  const int n = lane & 15;
  const int32_t* rec = tiles + (size_t)tile * 17;
  const int l = rec[0];
  const LevelDev lv1 = lvs[l - 1];
  const LevelDev lv2 = lvs[l - 2];
  gptr<int32_t> rank1 = as_global(lv1.rank);
  gptr<double> mass1 = as_global(lv1.mass);
  gptr<T> S1 = as_global(level_S<T>(lv1));
  gmut<T> part = as_global_mut((T*)lv1.part) + (size_t)chunk * lv1.nref * 32;
  if (lane < 16) sF[lane] = rec[1 + lane];
  __syncthreads();
  gptr<int32_t> refcell1 = as_global(lv1.refcell);
  gptr<int32_t> nbr2 = as_global(lv2.nbr);
  gptr<int32_t> rank2 = as_global(lv2.rank);
  for (int i = lane; i < 16 * 27; i += 64) {
    const int c = i / 27, e = i - c * 27;
    const int F = sF[c];
    int v = -1;
    if (F >= 0) {
      const int Q = nbr2[(size_t)(refcell1[F] >> 3) * 27 + e];
      if (Q >= 0) {
        const int rQ = rank2[Q];
        if (rQ >= 0) v = 8 * rQ;
      }
    }
    sCB[i] = v;
  }
  const int oF = refcell1[sF[0]] & 7;
  const int32_t* tpg = taps + oF * kTaps + tb;
  int off0[ST0], off1[ST1];
#pragma unroll
  for (int kb = 0; kb < ST0; ++kb) off0[kb] = aoff[kb * 64 + lane];
#pragma unroll
  for (int kb = 0; kb < ST1; ++kb) off1[kb] = aoff[(ST0 + kb) * 64 + lane];
  __syncthreads();
  // sources of every tap of the range
  const int nt = te - tb;
  const int32_t* tp = tpg;
  if constexpr (!XB) {
    for (int i = lane; i < nt * 16; i += 64) sSrcT[i] = tap_src(tp[i >> 4], i & 15, sCB, rank1);
    __syncthreads();
  }
  const int zrow = lv1.nref;
  V vD[ND];
  typename Acc4<T>::type acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
  // Taps run in pairs; an odd range ends with one empty tap (no source, so B
  // is zero; the D~ stage repeats the last tap's finite rows), so that both
  // halves of a pair and every load run unconditionally.
  const int nt2 = (nt + 1) & ~1;
  if constexpr (XB && P >= 6) {
    // One set of source rows in flight (tap k + 1, loaded row by row) and one
    // set of fragments in use (tap k): after tap k's MFMAs the rows of tap
    // k + 1, loaded a whole tap earlier, pass over the crossbar into the
    // fragments, so no MFMA waits on the crossbar.  No source table: each
    // lane resolves the two sources it needs (column xrow for its row loads,
    // column n for the monopole slot) two taps ahead, the rank lookup being
    // a load that lands while a tap runs; the block's LDS is then small
    // enough for 4 waves per SIMD.
    const int xrow = lane >> 2, xa = 4 * (4 * n + (lane >> 4));
    V braw[NV];
    T frag[ST0];
    auto cell_of = [&](int code, int col) {
      const int cb = sCB[col * 27 + (code & 31)];
      return cb < 0 ? -1 : cb + ((code >> 5) & 7);
    };
    // source code of a column (as tap_src) from its cell and rank, or -1
    // past the range
    auto fin = [](bool valid, int c, int rk) { return !valid || c < 0 ? -1 : (rk >= 0 ? rk : -2 - c); };
    // tap k + 1: cells and rank loads in flight; tap k + 2 likewise
    int cR1, cC1, kR1, kC1, cR2, cC2, kR2, kC2;
    auto resolve = [&](int k, int& cR, int& cC, int& kR, int& kC) {
      const int code = tp[k < nt ? k : nt - 1];
      cR = cell_of(code, xrow);
      cC = cell_of(code, n);
      kR = rank1[cR >= 0 ? cR : 0];
      kC = rank1[cC >= 0 ? cC : 0];
    };
    auto load_rows = [&](int srow, int scol, double& vm) {
      load_brows_xb<T, P, ST0>(srow, zrow, S1, braw);
      vm = mass1[scol <= -2 ? -2 - scol : 0];  // unconditional (a select on it would wait)
    };
    auto take = [&](int sr, double vm) {
#pragma unroll
      for (int kb = 0; kb < ST0; ++kb) frag[kb] = xb_take(xa, braw[kb / TS::VW][kb % TS::VW]);
      frag[0] = bfrag_m0<T>(sr, vm, frag[0]);
    };
    {
      int cR0, cC0, kR0, kC0;
      resolve(0, cR0, cC0, kR0, kC0);
      const int sc0 = fin(true, cC0, kC0);
      double vm0;
      load_rows(fin(true, cR0, kR0), sc0, vm0);
      load_dstage<T, P, 64>(tp[0], Dst, vD);
      resolve(1, cR1, cC1, kR1, kC1);
      store_dstage<T, P, 64>(sD[0], vD);
      take(sc0, vm0);
    }
    __syncthreads();
    auto step = [&](int k, int b) {
      const bool v1 = k + 1 < nt;
      const int srn = fin(v1, cC1, kC1);
      const int srr = fin(v1, cR1, kR1);
      load_dstage<T, P, 64>(tp[v1 ? k + 1 : nt - 1], Dst, vD);
      double vmn;
      load_rows(srr, srn, vmn);
      resolve(k + 2, cR2, cC2, kR2, kC2);
      __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the MFMAs
      const T* D = sD[b];
#pragma unroll
      for (int kb = 0; kb < ST0; ++kb) {
        acc0 = mfma16(D[off0[kb]], frag[kb], acc0);
        if (kb < ST1) acc1 = mfma16(D[off1[kb]], frag[kb], acc1);
      }
      __builtin_amdgcn_sched_barrier(0);  // the next fragments after the MFMAs
      take(srn, vmn);
      store_dstage<T, P, 64>(sD[b ^ 1], vD);
      cR1 = cR2, cC1 = cC2, kR1 = kR2, kC1 = kC2;
      __syncthreads();
    };
    for (int k = 0; k < nt2; k += 2) {
      step(k, 0);
      step(k + 1, 1);
    }
  } else if constexpr (XB) {
    // Short taps (p <= 5): the same crossbar form with source rows and D~
    // stages loaded two taps ahead (set k & 1 holds tap k's) and the sources
    // resolved three taps ahead, so that a load has two taps of MFMAs to land.
    const int xrow = lane >> 2, xa = 4 * (4 * n + (lane >> 4));
    V braw[2][NV];
    V vD2[2][ND];
    T frag[ST0];
    double vm[2];
    int sc[2];
    auto cell_of = [&](int code, int col) {
      const int cb = sCB[col * 27 + (code & 31)];
      return cb < 0 ? -1 : cb + ((code >> 5) & 7);
    };
    auto fin = [](bool valid, int c, int rk) { return !valid || c < 0 ? -1 : (rk >= 0 ? rk : -2 - c); };
    int cR, cC, kR, kC;  // the next tap to load: cells and rank loads in flight
    auto resolve = [&](int k) {
      const int code = tp[k < nt ? k : nt - 1];
      cR = cell_of(code, xrow);
      cC = cell_of(code, n);
      kR = rank1[cR >= 0 ? cR : 0];
      kC = rank1[cC >= 0 ? cC : 0];
    };
    // tap k into set q (sources from the pending resolution), then resolve k + 1
    auto prefetch = [&](int k, int q) {
      const bool v = k < nt;
      const int srr = fin(v, cR, kR);
      sc[q] = fin(v, cC, kC);
      load_dstage<T, P, 64>(tp[v ? k : nt - 1], Dst, vD2[q]);
      load_brows_xb<T, P, ST0>(srr, zrow, S1, braw[q]);
      vm[q] = mass1[sc[q] <= -2 ? -2 - sc[q] : 0];  // unconditional (a select on it would wait)
      resolve(k + 1);
    };
    auto take = [&](int q) {
#pragma unroll
      for (int kb = 0; kb < ST0; ++kb) frag[kb] = xb_take(xa, braw[q][kb / TS::VW][kb % TS::VW]);
      frag[0] = bfrag_m0<T>(sc[q], vm[q], frag[0]);
    };
    resolve(0);
    prefetch(0, 0);
    prefetch(1, 1);
    store_dstage<T, P, 64>(sD[0], vD2[0]);
    take(0);
    __syncthreads();
    // tap k (stage sD[b], set b): prefetch tap k + 2 into set b, MFMAs of tap
    // k, then tap k + 1 (set b ^ 1) into the fragments and the other stage
    auto step = [&](int k, int b) {
      prefetch(k + 2, b);
      __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the MFMAs
      const T* D = sD[b];
#pragma unroll
      for (int kb = 0; kb < ST0; ++kb) {
        acc0 = mfma16(D[off0[kb]], frag[kb], acc0);
        if (kb < ST1) acc1 = mfma16(D[off1[kb]], frag[kb], acc1);
      }
      __builtin_amdgcn_sched_barrier(0);  // the next fragments after the MFMAs
      take(b ^ 1);
      store_dstage<T, P, 64>(sD[b ^ 1], vD2[b ^ 1]);
      __syncthreads();
    };
    for (int k = 0; k < nt2; k += 2) {
      step(k, 0);
      step(k + 1, 1);
    }
  } else {
    V bA[NV], bB[NV];
    double vmA = 0, vmB = 0;
    int srA = sSrcT[n], srB = -1;
    load_bfrag_nb<T, P, ST0>(srA, zrow, mass1, S1, bA, vmA);
    load_dstage<T, P, 64>(tp[0], Dst, vD);
    store_dstage<T, P, 64>(sD[0], vD);
    __syncthreads();
    // one tap: prefetch tap k + 1 (D~ rows into vD, B into bn), MFMAs of tap k
    // from bc and the LDS stage sD[b]
    auto step = [&](int k, int b, const V* bc, int src, double vmc, V* bn, int& srn, double& vmn) {
      const int k1 = k + 1 < nt ? k + 1 : nt - 1;
      load_dstage<T, P, 64>(tp[k1], Dst, vD);
      srn = k + 1 < nt ? sSrcT[k1 * 16 + n] : -1;
      load_bfrag_nb<T, P, ST0>(srn, zrow, mass1, S1, bn, vmn);
      __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the MFMAs
      const T* D = sD[b];
#pragma unroll
      for (int kb = 0; kb < ST0; ++kb) {
        const T bv = kb == 0 ? bfrag_m0<T>(src, vmc, bc[0][0]) : bc[kb / TS::VW][kb % TS::VW];
        acc0 = mfma16(D[off0[kb]], bv, acc0);
        if (kb < ST1) acc1 = mfma16(D[off1[kb]], bv, acc1);
      }
      store_dstage<T, P, 64>(sD[b ^ 1], vD);
      __syncthreads();
    };
    for (int k = 0; k < nt2; k += 2) {
      step(k, 0, bA, srA, vmA, bB, srB, vmB);
      step(k + 1, 1, bB, srB, vmB, bA, srA, vmA);
    }
  }
  const int F = sF[n];
  if (F >= 0) {
    gmut<T> out = part + (size_t)F * 32;
    const int krow = lane >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = acc_row<T>(krow, r);
      out[i] = i < 8 ? acc0[r] : -acc0[r];
      out[16 + i] = -acc1[r];
    }
  }
}

// M2P with the source rows staged through LDS, for NT 16-column tiles per wave
// (tile shapes 1 and 2 of the launcher; the kernel above is shape 0).  In the
// direct form each lane's B fragments come from one of 16 source rows, so a
// 16-byte load of the wave touches 64 cache lines and the texture addresser
// and L1 tag lookups bound the kernel when a tap carries few MFMAs (low p).
// Here consecutive lanes load consecutive 16-byte pieces of a row (piece
// v = 64 j + lane is piece v % NVR of row v / NVR of the tap's 16 NT rows),
// two taps ahead; halfway through a tap's MFMAs the rows of the next tap go
// to an LDS row stage (padded by one vector per row: conflict-free fragment
// reads) and come back as MFMA fragments.  With NT = 2 one wave runs two
// tiles of the same parity class: each A fragment read from LDS feeds two
// MFMAs and one D~ stage serves 32 groups.  The block is one wave, whose LDS
// accesses complete in issue order, so the stages need no barrier.  The
// sources are resolved in chunks of CH taps; the code and sources of a tap
// are read from LDS one step before the loads that use them.
template <int NT>
constexpr int m2p_chunk() { return NT == 1 ? 64 : 32; }

template <typename T, int P, int NT>
__global__ __launch_bounds__(64) void k_m2p_s(const int32_t* __restrict__ tiles, int ntiles, int nsplit,
                                              const int32_t* __restrict__ taps, const int16_t* __restrict__ aoff,
                                              const LevelDev* __restrict__ lvs, const T* __restrict__ Dst) {
  using TS = TapStage<T, P>;
  using V = typename Vec16<T>::type;
  constexpr int K1 = nmi(P - 1);
  constexpr int ST0 = TS::KP / 4, ST1 = ((K1 + 3) & ~3) / 4;
  constexpr int NV = (ST0 + TS::VW - 1) / TS::VW;  // B vectors per lane and tile (MFMA layout)
  constexpr int ND = (TS::NDV + 63) / 64;
  constexpr int NC = 16 * NT;                      // groups (columns) of the block
  constexpr int NVR = TS::ROW / TS::VW;             // 16-byte pieces of a source row
  constexpr int RP = TS::ROW + TS::VW;              // LDS row stride
  constexpr int NG = (NC * NVR + 63) / 64;          // row pieces per lane and tap
  constexpr int CH = m2p_chunk<NT>();
  constexpr int KMID = ST0 / 2;
  static_assert(4 * NV <= NVR, "fragments inside the row");
  __shared__ __align__(16) T sD[2][TS::SDP];
  __shared__ __align__(16) T sB[NC * RP];
  __shared__ int sF[NC];
  __shared__ int sCB[NC * 27];
  __shared__ int sCode[kTaps];
  __shared__ int sSrc[CH * NC];
  const int item = xcd_tile(ntiles * nsplit);
  if (item >= ntiles * nsplit) return;
  const int tile = item / nsplit, chunk = item - tile * nsplit;
  int tb, te;
  tap_range(chunk, nsplit, tb, te);
  const int lane = threadIdx.x;
  const int n = lane & 15, g = lane >> 4;
  const int32_t* rec = tiles + (size_t)tile * (NC + 1);
  const int l = rec[0];
  const LevelDev lv1 = lvs[l - 1];
  const LevelDev lv2 = lvs[l - 2];
  gptr<int32_t> rank1 = as_global(lv1.rank);
  gptr<double> mass1 = as_global(lv1.mass);
  gptr<T> S1 = as_global(level_S<T>(lv1));
  gmut<T> part = as_global_mut((T*)lv1.part) + (size_t)chunk * lv1.nref * 32;
  if (lane < NC) sF[lane] = rec[1 + lane];
  __syncthreads();
  gptr<int32_t> refcell1 = as_global(lv1.refcell);
  gptr<int32_t> nbr2 = as_global(lv2.nbr);
  gptr<int32_t> rank2 = as_global(lv2.rank);
  for (int i = lane; i < NC * 27; i += 64) {
    const int c = i / 27, e = i - c * 27;
    const int F = sF[c];
    int v = -1;
    if (F >= 0) {
      const int Q = nbr2[(size_t)(refcell1[F] >> 3) * 27 + e];
      if (Q >= 0) {
        const int rQ = rank2[Q];
        if (rQ >= 0) v = 8 * rQ;
      }
    }
    sCB[i] = v;
  }
  const int oF = refcell1[sF[0]] & 7;
  const int32_t* tpg = taps + oF * kTaps + tb;
  const int nt = te - tb;
  for (int i = lane; i < nt; i += 64) sCode[i] = tpg[i];
  int off0[ST0], off1[ST1];
#pragma unroll
  for (int kb = 0; kb < ST0; ++kb) off0[kb] = aoff[kb * 64 + lane];
#pragma unroll
  for (int kb = 0; kb < ST1; ++kb) off1[kb] = aoff[(ST0 + kb) * 64 + lane];
  const int zrow = lv1.nref;
  // the row (0 .. NC-1) and piece of each of this lane's row pieces; pieces
  // past the last row re-read the last piece and are not stored
  int prow[NG], pchk[NG];
#pragma unroll
  for (int j = 0; j < NG; ++j) {
    const int v = min(64 * j + lane, NC * NVR - 1);
    prow[j] = v / NVR;
    pchk[j] = v - prow[j] * NVR;
  }
  typename Acc4<T>::type acc0[NT], acc1[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc0[t] = acc1[t] = {0, 0, 0, 0};
  // fragments (per tile) of the current and the next tap, row pieces of the
  // next two taps, and each tile's column source and mass for the monopole slot
  V bA[NT][NV], bB[NT][NV];
  V gX[NG], gY[NG];
  V vD[ND];
  double vmA[NT], vmB[NT], vmX[NT], vmY[NT];
  int srA[NT], srB[NT], srX[NT], srY[NT];
  int cN = 0, sN[NT], rN[NG];
#pragma unroll
  for (int t = 0; t < NT; ++t) vmA[t] = vmB[t] = vmX[t] = vmY[t] = 0, srA[t] = srB[t] = srX[t] = srY[t] = sN[t] = -1;
  auto load_rows = [&](const int* rs, V* gb) {
#pragma unroll
    for (int j = 0; j < NG; ++j) {
      const int row = rs[j] >= 0 ? rs[j] : zrow;
      gb[j] = *(gptr<V>)(S1 + (size_t)row * TS::ROW + pchk[j] * TS::VW);
    }
  };
  auto store_rows = [&](const V* gb) {
#pragma unroll
    for (int j = 0; j < NG; ++j)
      if (64 * j + lane < NC * NVR) *(V*)(sB + prow[j] * RP + pchk[j] * TS::VW) = gb[j];
  };
  auto read_frags = [&](V (*b)[NV]) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int j = 0; j < NV; ++j) b[t][j] = *(const V*)(sB + (16 * t + n) * RP + (4 * j + g) * TS::VW);
  };
  // the mass of a leaf source for lane group 0 (the only lanes that use it)
  auto load_mass = [&](const int* sr, double* vm) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      double v = 0;
      if (g == 0 && sr[t] <= -2) v = mass1[-2 - sr[t]];
      vm[t] = v;
    }
  };
  // sources of chunk tap k (none past the chunk): columns of this lane, rows of its pieces
  auto read_srcs = [&](int k, int cn) {
#pragma unroll
    for (int t = 0; t < NT; ++t) sN[t] = k < cn ? sSrc[k * NC + 16 * t + n] : -1;
#pragma unroll
    for (int j = 0; j < NG; ++j) rN[j] = k < cn ? sSrc[k * NC + prow[j]] : -1;
  };
  for (int c0 = 0; c0 < nt; c0 += CH) {
    const int cn = min(CH, nt - c0);
    __syncthreads();
    for (int i = lane; i < cn * NC; i += 64) sSrc[i] = tap_src(sCode[c0 + i / NC], i % NC, sCB, rank1);
    __syncthreads();
    {
      // tap 0 into the stages and bA; tap 1's rows in flight (set X); tap 2's sources read
      read_srcs(0, cn);
      load_rows(rN, gY);
#pragma unroll
      for (int t = 0; t < NT; ++t) srA[t] = sN[t];
      load_mass(srA, vmA);
      load_dstage<T, P, 64>(sCode[c0], Dst, vD);
      store_dstage<T, P, 64>(sD[0], vD);
      store_rows(gY);
      read_frags(bA);
      read_srcs(1, cn);
      load_rows(rN, gX);
#pragma unroll
      for (int t = 0; t < NT; ++t) srX[t] = sN[t];
      load_mass(srX, vmX);
      cN = sCode[c0 + (cn > 1 ? 1 : 0)];
      read_srcs(2, cn);
    }
    __builtin_amdgcn_wave_barrier();
    // step k: rows of tap k + 2 into gn (sources read one step ago) and the D~
    // stage of tap k + 1 into vD; the MFMAs of tap k, halfway through them the
    // rows of tap k + 1 (gc) through the LDS row stage into bn; then the D~
    // stage of tap k + 1 into LDS.  Taps run in pairs; an odd chunk ends with
    // one empty tap (zero rows; its D~ stage repeats the last tap's rows).
    auto step = [&](int k, int b, V (*bc)[NV], const int* srcc, const double* vmc, V (*bn)[NV], int* srn,
                    double* vmn, const V* gc, const int* src1, const double* vm1, V* gn, int* sr2, double* vm2) {
      load_dstage<T, P, 64>(cN, Dst, vD);
      load_rows(rN, gn);
#pragma unroll
      for (int t = 0; t < NT; ++t) sr2[t] = sN[t];
      load_mass(sr2, vm2);
      cN = sCode[c0 + (k + 2 < cn ? k + 2 : cn - 1)];
      read_srcs(k + 3, cn);
      __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the MFMAs
      const T* D = sD[b];
#pragma unroll
      for (int kb = 0; kb < ST0; ++kb) {
        const T a0 = D[off0[kb]];
        const T a1 = kb < ST1 ? D[off1[kb]] : (T)0;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const T bv = kb == 0 ? bfrag_m0<T>(srcc[t], vmc[t], bc[t][0][0]) : bc[t][kb / TS::VW][kb % TS::VW];
          acc0[t] = mfma16(a0, bv, acc0[t]);
          if (kb < ST1) acc1[t] = mfma16(a1, bv, acc1[t]);
        }
        if (kb == KMID) {
          store_rows(gc);
          read_frags(bn);
#pragma unroll
          for (int t = 0; t < NT; ++t) srn[t] = src1[t], vmn[t] = vm1[t];
        }
      }
      store_dstage<T, P, 64>(sD[b ^ 1], vD);
      __builtin_amdgcn_wave_barrier();
    };
    const int cn2 = (cn + 1) & ~1;
    for (int k = 0; k < cn2; k += 2) {
      step(k, 0, bA, srA, vmA, bB, srB, vmB, gX, srX, vmX, gY, srY, vmY);
      step(k + 1, 1, bB, srB, vmB, bA, srA, vmA, gY, srY, vmY, gX, srX, vmX);
    }
  }
  const int krow = lane >> 4;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int F = sF[16 * t + n];
    if (F < 0) continue;
    gmut<T> out = part + (size_t)F * 32;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = acc_row<T>(krow, r);
      out[i] = i < 8 ? acc0[t][r] : -acc0[t][r];
      out[16 + i] = -acc1[t][r];
    }
  }
}

// ---------------------------------------------------------------------------
// M2L tap sums at the FMM levels (Alg. 3 without the ShiftLocal term, which
// the L2L chain adds afterwards): rows R = 8 b + o (local coefficient b, child
// octant o; b in degree order, so 16-row tile T starts at coefficient 2T and
// needs only the first ks(T)*4 multipole coefficients: the triangle
// |a|+|b| <= p), columns = 16 groups.  The row tiles are split over the 4
// waves by a compile-time greedy balance of their k-steps; each wave runs a
// fully unrolled MFMA sequence with its A offsets in registers.
constexpr int deg_of(int idx) {
  int n = 0;
  while (nmi(n) <= idx) ++n;
  return n;
}
constexpr int m2l_ksteps(int P, int T) { return (nmi(P - deg_of(2 * T)) + 3) / 4; }

template <int P>
struct M2LPlan {
  static constexpr int NT = (8 * nmi(P) + 15) / 16;
  int n[4] = {0, 0, 0, 0};
  int tile[4][NT] = {};
  int steps[4] = {0, 0, 0, 0};
  int kbmax[4] = {0, 0, 0, 0};
  int base[NT] = {};   // first step of tile T in the natural-order offset table
};

template <int P>
constexpr M2LPlan<P> make_m2l_plan() {
  M2LPlan<P> pl{};
  constexpr int NT = M2LPlan<P>::NT;
  int s = 0;
  for (int T = 0; T < NT; ++T) {
    pl.base[T] = s;
    s += m2l_ksteps(P, T);
  }
  // tiles in natural order have non-increasing k-steps: greedy to the lightest part
  for (int T = 0; T < NT; ++T) {
    int best = 0;
    for (int q = 1; q < 4; ++q)
      if (pl.steps[q] < pl.steps[best]) best = q;
    pl.tile[best][pl.n[best]++] = T;
    pl.steps[best] += m2l_ksteps(P, T);
    if (m2l_ksteps(P, T) > pl.kbmax[best]) pl.kbmax[best] = m2l_ksteps(P, T);
  }
  return pl;
}

// B of one M2L tap in LDS, fragment order sB[kb][lane]: wave w loads vectors
// j in [w NVW, (w+1) NVW) of every lane's run (16-byte loads) and writes
// element e of vector j to sB[(VW j + e) * 64 + lane] (consecutive lanes,
// consecutive banks).
template <typename T, int P>
struct M2LStage {
  static constexpr int NVB = TapStage<T, P>::STP / TapStage<T, P>::VW;  // vectors per lane run
  static constexpr int NVW = (NVB + 3) / 4;                            // per wave
};

// Wave w's share of the B stage of a tap (vectors j in [w NVW, (w+1) NVW) of
// every lane's run).  Branch-free: a missing or leaf source reads the zero
// row zrow of the source copy, and wave 0 also loads a mass (cell 0 when the
// source is no leaf) that store_bshare puts into the monopole slot.
template <typename T, int P, int W>
__device__ inline void load_bshare(int sr, int zrow, int lane, gptr<double> mass1, gptr<T> S1,
                                   typename Vec16<T>::type* vb, double& vm) {
  using TS = TapStage<T, P>;
  using MS = M2LStage<T, P>;
  using V = typename Vec16<T>::type;
  gptr<T> src = S1 + (size_t)(sr >= 0 ? sr : zrow) * TS::ROW;
#pragma unroll
  for (int i = 0; i < MS::NVW; ++i) {
    constexpr int j0 = W * MS::NVW;
    if (j0 + i < MS::NVB) vb[i] = *(gptr<V>)(src + src_vec(j0 + i, lane >> 4, (int)sizeof(T)));
  }
  if (W == 0) vm = mass1[sr <= -2 ? -2 - sr : 0];
}

template <typename T, int P, int W>
__device__ inline void store_bshare(T* sB, int sr, int lane, typename Vec16<T>::type* vb, double vm) {
  using TS = TapStage<T, P>;
  using MS = M2LStage<T, P>;
  if (W == 0 && sr <= -2 && (lane >> 4) == 0) vb[0][0] = (T)vm;
#pragma unroll
  for (int i = 0; i < MS::NVW; ++i) {
    const int j = W * MS::NVW + i;
    if (j < MS::NVB) {
#pragma unroll
      for (int e = 0; e < TS::VW; ++e) sB[(j * TS::VW + e) * 64 + lane] = vb[i][e];
    }
  }
}

// D~ stage copy without a branch around the loads: thread t loads vectors
// t, t + NTH, ... clamped to the last one (stores skip the extra ones).
template <typename T, int P, int NTH>
__device__ inline void load_dstage_nb(int code, const T* __restrict__ Dst, typename Vec16<T>::type* vD) {
  using TS = TapStage<T, P>;
  using V = typename Vec16<T>::type;
  constexpr int NJ = (TS::NDV + NTH - 1) / NTH;
  const int t = threadIdx.x;
  gptr<V> src = (gptr<V>)as_global(Dst + (size_t)(code >> 8) * TS::SDP);
#pragma unroll
  for (int j = 0; j < NJ; ++j) vD[j] = src[min(t + NTH * j, TS::NDV - 1)];
}

// One wave's share of an M2L tile: its row tiles (compile-time plan H) over
// the block's LDS stage of B and of the D~ rows.  The stage of tap k + 2 is
// loaded into registers while the MFMAs of tap k run and stored to LDS after
// those of tap k + 1 (two register sets, two LDS buffers), so a load has two
// taps to land; the sources of every tap of the range were resolved into LDS
// (sSrcT) before the loop.
template <typename T, int P, int H>
__device__ inline void m2l_part(const int32_t* __restrict__ tp, int nt, const int16_t* __restrict__ aoff,
                                const int* sF, const int* sSrcT, T (*sB)[TapStage<T, P>::STP * 64],
                                T (*sD)[TapStage<T, P>::SDP], int zrow, gptr<double> mass1,
                                const T* __restrict__ Dst, gptr<T> S1, gptr<int32_t> rank0, gmut<T> Lout) {
  using TS = TapStage<T, P>;
  using MS = M2LStage<T, P>;
  using V = typename Vec16<T>::type;
  constexpr int K = TS::K;
  constexpr M2LPlan<P> PL = make_m2l_plan<P>();
  constexpr int NTH = PL.n[H];
  constexpr int NS = PL.steps[H];
  constexpr int KBH = PL.kbmax[H];
  constexpr int ND = (TS::NDV + kBlock - 1) / kBlock;
  const int t = threadIdx.x, lane = t & 63, krow = lane >> 4, n = lane & 15;
  int off[NS > 0 ? NS : 1];
  {
    int s = 0;
#pragma unroll
    for (int i = 0; i < NTH; ++i)
#pragma unroll
      for (int kb = 0; kb < m2l_ksteps(P, PL.tile[H][i]); ++kb) off[s++] = aoff[(PL.base[PL.tile[H][i]] + kb) * 64 + lane];
  }
  typename Acc4<T>::type acc[NTH > 0 ? NTH : 1];
#pragma unroll
  for (int i = 0; i < NTH; ++i) acc[i] = {0, 0, 0, 0};
  // register sets X (odd taps ahead) and Y; tap 1 goes to X first
  V vDX[ND], vDY[ND], vBX[MS::NVW], vBY[MS::NVW];
  double vmX = 0, vmY = 0;
  int srX = -1, srY = -1;
  // Taps run in pairs; an odd range ends with one empty tap (no source, so B
  // is zero; its D~ stage repeats the last tap's finite rows), so that both
  // steps of a pair and every load run unconditionally.
  const int nt2 = (nt + 1) & ~1;
  {
    const int k1 = nt > 1 ? 1 : 0;
    srX = nt > 1 ? sSrcT[16 + n] : -1;
    load_dstage_nb<T, P, kBlock>(tp[k1], Dst, vDX);
    load_bshare<T, P, H>(srX, zrow, lane, mass1, S1, vBX, vmX);
  }
  // one tap: load tap k + 2 into (vDn, vBn), MFMAs of tap k from LDS buffer
  // b, store tap k + 1 from (vDc, vBc) into buffer b ^ 1
  auto step = [&](int k, int b, V* vDc, V* vBc, double vmc, int src, V* vDn, V* vBn, double& vmn, int& srn) {
    const int k2 = k + 2 < nt ? k + 2 : nt - 1;
    srn = k + 2 < nt ? sSrcT[k2 * 16 + n] : -1;
    load_dstage_nb<T, P, kBlock>(tp[k2], Dst, vDn);
    load_bshare<T, P, H>(srn, zrow, lane, mass1, S1, vBn, vmn);
    __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the MFMAs
    const T* B = sB[b] + lane;
    const T* D = sD[b];
    T bv[KBH > 0 ? KBH : 1];
#pragma unroll
    for (int kb = 0; kb < KBH; ++kb) bv[kb] = B[kb * 64];
    int s = 0;
#pragma unroll
    for (int i = 0; i < NTH; ++i)
#pragma unroll
      for (int kb = 0; kb < m2l_ksteps(P, PL.tile[H][i]); ++kb) {
        acc[i] = mfma16(D[off[s]], bv[kb], acc[i]);
        ++s;
      }
    if (k + 1 < nt2) {
      store_dstage<T, P, kBlock>(sD[b ^ 1], vDc);
      store_bshare<T, P, H>(sB[b ^ 1], src, lane, vBc, vmc);
    }
    __syncthreads();
  };
  for (int k = 0; k < nt2; k += 2) {
    step(k, 0, vDX, vBX, vmX, srX, vDY, vBY, vmY, srY);
    step(k + 1, 1, vDY, vBY, vmY, srY, vDX, vBX, vmX, srX);
  }
  const int F = sF[lane & 15];
  if (F < 0) return;
#pragma unroll
  for (int i = 0; i < NTH; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int R = 16 * PL.tile[H][i] + acc_row<T>(krow, r);
      if ((R >> 3) >= K) continue;
      const int ry = rank0[8 * F + (R & 7)];
      if (ry >= 0) Lout[(size_t)ry * K + (R >> 3)] = acc[i][r];
    }
  }
}

// Occupancy floor of k_m2l_mfma: for FP32 up to p = 6 the kernel fits 128
// registers without spilling, so its LDS (4 blocks per CU) sets 4 waves per
// SIMD; left to itself the compiler takes about 176 registers and 2 waves,
// and the M2L launches ran about 8% slower.  At p = 8 (FP32) a floor of 2
// waves (256 registers, 20 bytes of spill, against 348 registers and 1 wave)
// ran 28% faster.  Other instantiations keep the compiler's choice (p = 7
// already runs 2 waves, and a floor of 3 spills; FP64 spills at any floor that
// would raise its occupancy).
template <typename T, int P>
constexpr int m2l_min_waves() { return sizeof(T) != 4 ? 1 : P <= 6 ? 4 : P == 8 ? 2 : 1; }

// One block = one tile (16 groups) and one of `nsplit` contiguous tap ranges.
// With nsplit == 1 the sums go straight to L; otherwise to the level's
// partial buffer [nsplit][nref][K], reduced in fixed order by k_l2l.
template <typename T, int P>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(m2l_min_waves<T, P>())))
void k_m2l_mfma(const int32_t* __restrict__ tiles, int ntiles, int nsplit,
                                                     const int32_t* __restrict__ taps,
                                                     const int16_t* __restrict__ aoff,
                                                     const LevelDev* __restrict__ lvs, const T* __restrict__ Dst) {
  using TS = TapStage<T, P>;
  using MS = M2LStage<T, P>;
  constexpr int ND = (TS::NDV + kBlock - 1) / kBlock;
  __shared__ T sB[2][TS::STP * 64];
  __shared__ __align__(16) T sD[2][TS::SDP];
  __shared__ int sF[16];
  __shared__ int sCB[16 * 27];
  __shared__ int sSrcT[kTaps * 16];
  __shared__ int sCode[kTaps];
  __shared__ int sNt;
  const int item = xcd_tile(ntiles * nsplit);
  if (item >= ntiles * nsplit) return;
  const int tile = item / nsplit, chunk = item - tile * nsplit;
  int tb, te;
  tap_range(chunk, nsplit, tb, te);
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int32_t* rec = tiles + (size_t)tile * 17;
  const int f = rec[0];
  const LevelDev lv1 = lvs[f - 1];
  const LevelDev lv0 = lvs[f];
  tile_setup(rec, 16, lvs[f - 2], lv1, sF, sCB);
  __syncthreads();
  const int oF = as_global(lv1.refcell)[sF[0]] & 7;
  const int32_t* tpg = taps + oF * kTaps + tb;
  gptr<T> S1 = as_global(level_S<T>(lv1));
  gptr<int32_t> rank1 = as_global(lv1.rank);
  gptr<double> mass1 = as_global(lv1.mass);
  // sources of every tap of the range, then the taps with a source (wave 0)
  for (int i = t; i < (te - tb) * 16; i += kBlock) sSrcT[i] = tap_src(tpg[i >> 4], i & 15, sCB, rank1);
  __syncthreads();
  if (w == 0) {
    const int c = compact_taps(te - tb, tpg, sSrcT, sCode);
    if (lane == 0) sNt = c;
  }
  __syncthreads();
  const int nt = sNt;
  const int* tp = sCode;
  const int zrow = lv1.nref;
  {
    typename Vec16<T>::type vD[ND];
    typename Vec16<T>::type vB[MS::NVW];
    double vm = 0;
    const int sr = sSrcT[lane & 15];
    load_dstage_nb<T, P, kBlock>(tp[0], Dst, vD);
    switch (w) {
      case 0: load_bshare<T, P, 0>(sr, zrow, lane, mass1, S1, vB, vm); store_bshare<T, P, 0>(sB[0], sr, lane, vB, vm); break;
      case 1: load_bshare<T, P, 1>(sr, zrow, lane, mass1, S1, vB, vm); store_bshare<T, P, 1>(sB[0], sr, lane, vB, vm); break;
      case 2: load_bshare<T, P, 2>(sr, zrow, lane, mass1, S1, vB, vm); store_bshare<T, P, 2>(sB[0], sr, lane, vB, vm); break;
      default: load_bshare<T, P, 3>(sr, zrow, lane, mass1, S1, vB, vm); store_bshare<T, P, 3>(sB[0], sr, lane, vB, vm); break;
    }
    store_dstage<T, P, kBlock>(sD[0], vD);
  }
  __syncthreads();
  gmut<T> Lout = as_global_mut(nsplit > 1 ? (T*)lv0.Lpart + (size_t)chunk * lv0.nref * TS::K : level_L<T>(lv0));
  gptr<int32_t> rank0 = as_global(lv0.rank);
  // every wave runs the same number of barriers (one per tap)
  switch (w) {
    case 0: m2l_part<T, P, 0>(tp, nt, aoff, sF, sSrcT, sB, sD, zrow, mass1, Dst, S1, rank0, Lout); break;
    case 1: m2l_part<T, P, 1>(tp, nt, aoff, sF, sSrcT, sB, sD, zrow, mass1, Dst, S1, rank0, Lout); break;
    case 2: m2l_part<T, P, 2>(tp, nt, aoff, sF, sSrcT, sB, sD, zrow, mass1, Dst, S1, rank0, Lout); break;
    default: m2l_part<T, P, 3>(tp, nt, aoff, sF, sSrcT, sB, sD, zrow, mass1, Dst, S1, rank0, Lout); break;
  }
}

// ---------------------------------------------------------------------------
// Leaf evaluation at level l (Alg. 4): far field (L2P of L[F]) and near field
// (P2P from the level-l leaves among the children of F's 27 neighbours and
// from the neighbours that are leaves one level coarser).  For every group
// these are one fixed linear map of the same gathered inputs (the candidates'
// masses, L[F]), so 16 groups are one product [32 x near_cols] . [near_cols x
// 16] on 16x16x4 MFMA: rows c * 8 + o (phi, ax, ay, az of child o), columns
// in the order of the operator table nearA.  Lane (n = lane & 15, g = lane >>
// 4) gathers column n's inputs for steps 4 kb + g straight into registers.
// The intermediate-field partials (k_m2p) and the partial of the refined near
// cells (near M2P and nearest-field P2P, k_near_m2p; zero for groups without
// such cells) are added in FP64 and the sums scaled to physical units.  One
// block per 16 groups of the level's group list; its 4 waves take a quarter
// of the operator columns each (more loads in flight per tile), and wave 0
// adds the other waves' accumulators in order.
template <typename T, int P, int W>
__device__ inline void near_part(int lane, int F, const int* __restrict__ sCB, gptr<double> mass0,
                                 gptr<double> mass1, const T* __restrict__ Lpar, const T* __restrict__ nearA,
                                 typename Acc4<T>::type& acc0, typename Acc4<T>::type& acc1) {
  using V = typename Vec16<T>::type;
  constexpr int K = nmi(P);
  constexpr int VW = 16 / (int)sizeof(T);
  constexpr int NQ = near_ksteps(P) / VW;
  constexpr int Q0 = W * NQ / 4, Q1 = (W + 1) * NQ / 4;
  constexpr int C0 = kNearLeafCols, C1 = kNearLeafCols + kNearCoarseCols;
  const int n = lane & 15, g = lane >> 4;
  // B: column n's inputs for steps 4 kb + g (refined cells hold mass 0; every
  // load has a valid address, the value is selected afterwards)
  T bv[(Q1 - Q0) * VW + 1];
#pragma unroll
  for (int i = 0; i < (Q1 - Q0) * VW; ++i) {
    const int k = 4 * (Q0 * VW + i) + g;
    T v = 0;
    if (k < C0) {
      const int cb = sCB[n * 27 + (k >> 3)];
      const double m = mass0[cb >= 0 ? cb + (k & 7) : 0];
      v = cb >= 0 ? (T)m : (T)0;
    } else if (k < C1) {
      const int cb = sCB[n * 27 + (k - C0)];
      const double m = mass1[cb <= -2 ? -2 - cb : 0];
      v = cb <= -2 ? (T)m : (T)0;
    } else if (k < C1 + K) {
      if (Lpar) {
        const T l = as_global(Lpar)[(size_t)(F >= 0 ? F : 0) * K + (k - C1)];
        v = F >= 0 ? l : (T)0;
      }
    }
    bv[i] = v;
  }
  gptr<V> A = (gptr<V>)as_global(nearA);
#pragma unroll
  for (int q = Q0; q < Q1; ++q) {
    const V a0 = A[(size_t)q * 64 + lane];
    const V a1 = A[(size_t)(NQ + q) * 64 + lane];
#pragma unroll
    for (int j = 0; j < VW; ++j) {
      acc0 = mfma16(a0[j], bv[(q - Q0) * VW + j], acc0);
      acc1 = mfma16(a1[j], bv[(q - Q0) * VW + j], acc1);
    }
  }
}

template <typename T, int P>
__global__ __launch_bounds__(kBlock) void k_near(const int32_t* __restrict__ grp, int ngrp, LevelDev lv1, LevelDev lv0,
                                                 const T* __restrict__ nearA, const T* __restrict__ Lpar,
                                                 const T* __restrict__ part, const T* __restrict__ nmp, double G,
                                                 double h, double cself, double* __restrict__ phi,
                                                 double* __restrict__ acc) {
  static_assert(kBlock == 256, "four waves split the operator columns");
  static_assert(near_ksteps(P) % (16 / (int)sizeof(T)) == 0, "near operator vectors");
  __shared__ int sF[16];
  __shared__ int sCB[16 * 27];
  __shared__ T sAcc[3][8][64];
  const int ntiles = (ngrp + 15) / 16;
  const int tile = xcd_tile(ntiles);
  if (tile >= ntiles) return;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  if (t < 16) sF[t] = 16 * tile + t < ngrp ? grp[16 * tile + t] : -1;
  __syncthreads();
  // per group and neighbour e: child base 8 rq (refined neighbour), -2 - q
  // (leaf neighbour q), or -1 (outside the box)
  gptr<int32_t> nbr1 = as_global(lv1.nbr), rank1 = as_global(lv1.rank);
  for (int i = t; i < 16 * 27; i += kBlock) {
    const int c = i / 27, e = i - 27 * c;
    const int F = sF[c];
    int v = -1;
    if (F >= 0) {
      const int q = nbr1[(size_t)F * 27 + e];
      if (q >= 0) {
        const int rq = rank1[q];
        v = rq >= 0 ? 8 * rq : -2 - q;
      }
    }
    sCB[i] = v;
  }
  __syncthreads();
  const int n = lane & 15, g = lane >> 4;
  const int F = sF[n];
  gptr<double> mass0 = as_global(lv0.mass), mass1 = as_global(lv1.mass);
  typename Acc4<T>::type acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
  switch (w) {
    case 0: near_part<T, P, 0>(lane, F, sCB, mass0, mass1, Lpar, nearA, acc0, acc1); break;
    case 1: near_part<T, P, 1>(lane, F, sCB, mass0, mass1, Lpar, nearA, acc0, acc1); break;
    case 2: near_part<T, P, 2>(lane, F, sCB, mass0, mass1, Lpar, nearA, acc0, acc1); break;
    default: near_part<T, P, 3>(lane, F, sCB, mass0, mass1, Lpar, nearA, acc0, acc1); break;
  }
  if (w > 0)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      sAcc[w - 1][r][lane] = acc0[r];
      sAcc[w - 1][4 + r][lane] = acc1[r];
    }
  __syncthreads();
  if (w > 0 || F < 0) return;
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      acc0[r] += sAcc[v][r][lane];
      acc1[r] += sAcc[v][4 + r][lane];
    }
  gptr<int32_t> rank0 = as_global(lv0.rank), slot0 = as_global(lv0.slot);
  const double sp = G / h, sa = G / (h * h);
#pragma unroll
  for (int tt = 0; tt < 2; ++tt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int R = 16 * tt + acc_row<T>(g, r);
      const int c = R >> 3, cell = 8 * F + (R & 7);
      if (rank0[cell] >= 0) continue;  // refined child: not a target
      double v = (double)(tt ? acc1[r] : acc0[r]);
      if (part)
        for (int s = 0; s < lv1.npart; ++s) v += (double)as_global(part)[((size_t)s * lv1.nref + F) * 32 + R];
      if (nmp) v += (double)as_global(nmp)[(size_t)F * 32 + R];
      const int sl = slot0[cell];
      if (c == 0)
        phi[sl] = sp * (v - cself * mass0[cell]);  // optional self term of the leaf's own mass
      else
        acc[3 * (size_t)sl + c - 1] = sa * v;
    }
}

// Refined level-l cells among the near candidates of a group (children of
// F's 27 neighbours): M2P from those that do not touch the target (Alg. 4) and
// P2P from the 8 children of those that do (nearest field, Sec. 3.2; the
// children are leaves by the grading rule).  One block per group: the refined
// candidates are compacted into LDS (ballot per wave, in candidate order),
// thread (o = t & 7, j = t >> 3) takes target o and every 32nd candidate from
// j, first for the M2P and then, in a separate loop, for the nearest field
// (so that threads on one path do not wait for the other); partial sums are
// reduced by shuffles within a wave and in order across the waves, and
// threads 0..7 write nmp[F][c * 8 + o] (target-level units), read by k_near.
// Every child o is evaluated (refined ones are not read).
template <typename T, int P>
__global__ __launch_bounds__(kBlock) void k_near_m2p(const int32_t* __restrict__ grp, int ngrp, LevelDev lv1,
                                                     LevelDev lv0, LevelDev lvp, const T* __restrict__ Dsame,
                                                     const T* __restrict__ S0, T* __restrict__ nmp) {
  static_assert(kBlock == 256, "one candidate per thread in the compaction");
  constexpr int K = nmi(P);
  constexpr int NW = kBlock / 64;
  constexpr int NJ = kBlock / 8;
  __shared__ int s_c[216];
  __shared__ int s_rn[216];
  __shared__ int s_cnt[NW];
  __shared__ T s_red[NW][4][8];
  const int gi = blockIdx.x;
  if (gi >= ngrp) return;
  const int F = grp[gi];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  int rn = -1;
  if (t < 216) {
    const int q = lv1.nbr[(size_t)F * 27 + (t >> 3)];
    if (q >= 0) {
      const int rq = lv1.rank[q];
      if (rq >= 0) rn = lv0.rank[8 * rq + (t & 7)];
    }
  }
  const uint64_t m = __ballot(rn >= 0);
  if (lane == 0) s_cnt[w] = __popcll(m);
  __syncthreads();
  int base = 0, nlist = 0;
#pragma unroll
  for (int v = 0; v < NW; ++v) {
    base += v < w ? s_cnt[v] : 0;
    nlist += s_cnt[v];
  }
  if (rn >= 0) {
    const int pos = base + __popcll(m & ((1ull << lane) - 1ull));
    s_c[pos] = t;
    s_rn[pos] = rn;
  }
  __syncthreads();
  const int o = t & 7, j = t >> 3;
  T sum[4] = {0, 0, 0, 0};
  for (int i = j; i < nlist; i += NJ) {
    const int c = s_c[i], e = c >> 3, op = c & 7;
    const int tx = o_axis(o, 0) - 2 * e_axis(e, 0) - o_axis(op, 0);
    const int ty = o_axis(o, 1) - 2 * e_axis(e, 1) - o_axis(op, 1);
    const int tz = o_axis(o, 2) - 2 * e_axis(e, 2) - o_axis(op, 2);
    if (max(abs(tx), max(abs(ty), abs(tz))) <= 1) continue;
    m2p_row<T, P>(Dsame + (size_t)d_index(tx, ty, tz) * K, S0 + (size_t)s_rn[i] * src_row(P, (int)sizeof(T)), sum);
  }
  gptr<double> massp = as_global(lvp.mass);
  for (int i = j; i < nlist; i += NJ) {
    const int c = s_c[i], e = c >> 3, op = c & 7;
    const int tx = o_axis(o, 0) - 2 * e_axis(e, 0) - o_axis(op, 0);
    const int ty = o_axis(o, 1) - 2 * e_axis(e, 1) - o_axis(op, 1);
    const int tz = o_axis(o, 2) - 2 * e_axis(e, 2) - o_axis(op, 2);
    if (max(abs(tx), max(abs(ty), abs(tz))) > 1) continue;
    double mc[8];
#pragma unroll
    for (int o2 = 0; o2 < 8; ++o2) mc[o2] = massp[8 * s_rn[i] + o2];
#pragma unroll
    for (int o2 = 0; o2 < 8; ++o2)
      p2p<T>((T)tx - ((T)o_axis(o2, 0) - (T)0.5) * (T)0.5, (T)ty - ((T)o_axis(o2, 1) - (T)0.5) * (T)0.5,
             (T)tz - ((T)o_axis(o2, 2) - (T)0.5) * (T)0.5, (T)mc[o2], sum);
  }
#pragma unroll
  for (int d = 8; d <= 32; d <<= 1)
#pragma unroll
    for (int c = 0; c < 4; ++c) sum[c] += __shfl_xor(sum[c], d, 64);
  if (lane < 8)
#pragma unroll
    for (int c = 0; c < 4; ++c) s_red[w][c][o] = sum[c];
  __syncthreads();
  if (t < 8)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      T v = 0;
#pragma unroll
      for (int u = 0; u < NW; ++u) v += s_red[u][c][o];
      nmp[(size_t)F * 32 + c * 8 + o] = v;
    }
}

// Stale trees advanced to the solve's time: each slot's level is found by a
// scan of the (at most 21) level offsets.
__global__ void k_drift(DriftLevels d, const double* __restrict__ m, const double* __restrict__ rate,
                        double* __restrict__ out, int64_t nslots) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslots; s += (int64_t)gridDim.x * blockDim.x) {
    int i = 0;
    while (i + 1 < d.n && s >= d.off[i + 1]) ++i;
    const double dt = d.dt[i];
    out[s] = dt != 0.0 ? m[s] + dt * rate[s] : m[s];
  }
}

// ---------------------------------------------------------------------------
// launchers

hipError_t launch_drift(const DriftLevels& d, const double* m, const double* rate, double* out, int64_t nslots,
                        hipStream_t st) {
  if (nslots <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((nslots + 255) / 256, 8192);
  hipLaunchKernelGGL(k_drift, dim3(blocks), dim3(256), 0, st, d, m, rate, out, nslots);
  return hipGetLastError();
}

template <typename T>
static hipError_t m2p_dispatch(int p, const MfmaTiles& mt, int t0, int n, int nsplit, const MfmaTables& tabs,
                               const LevelDev* lvs, const T* Dst, int shape, hipStream_t st) {
  const int items = n * nsplit;
  const dim3 grid(8 * ((items + 7) / 8)), block(64);
  const int32_t* tl = mt.tiles + (size_t)t0 * (mt.nc + 1);
  if (!m2p_shape_ok(p, sizeof(T) == 4, shape) || mt.nc != m2p_shape_columns(shape)) return hipErrorInvalidValue;
  if (shape == 1 || shape == 2) {
    if constexpr (sizeof(T) == 4) {
      switch (p * 4 + shape) {
#define AFMM_M2PS(PP, SH)                                                                                      \
  case PP * 4 + SH:                                                                                           \
    hipLaunchKernelGGL((k_m2p_s<T, PP, SH>), grid, block, 0, st, tl, n, nsplit, tabs.taps, tabs.m2p_off, lvs, Dst); \
    break;
        AFMM_M2PS(1, 1) AFMM_M2PS(2, 1) AFMM_M2PS(3, 1) AFMM_M2PS(4, 1) AFMM_M2PS(5, 1) AFMM_M2PS(6, 1)
        AFMM_M2PS(7, 1) AFMM_M2PS(8, 1) AFMM_M2PS(1, 2) AFMM_M2PS(2, 2) AFMM_M2PS(3, 2) AFMM_M2PS(4, 2)
        AFMM_M2PS(5, 2)
#undef AFMM_M2PS
        default: return hipErrorInvalidValue;
      }
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  // LDS source table of k_m2p: the longest tap range of the split, except
  // for FP32 from p = 6 on, where the table keeps all 189 taps so that the
  // block's LDS (about 20 KB) holds the kernel at 2 waves per SIMD.  Measured:
  // FP32 at p = 6, 2 waves per SIMD beat 3 and 4 (the 16 source rows each wave
  // streams thrash L1 when more waves share it); FP32 at p = 4 (a short tap of
  // 14 MFMAs leaves the waits exposed) and FP64 at p = 6 ran 7-9% faster with
  // the smaller table at a split of 3.
  int ntmax = 0;
  for (int c = 0; c < nsplit; ++c) {
    int tb, te;
    tap_range(c, nsplit, tb, te);
    ntmax = std::max(ntmax, te - tb);
  }
  const size_t lds = shape == 3 ? 0 : (size_t)(sizeof(T) == 4 && p >= 6 ? kTaps : ntmax) * 16 * sizeof(int);
  switch (p * 2 + (shape == 3)) {
#define AFMM_M2P(PP, XB)                                                                                         \
  case PP * 2 + XB:                                                                                              \
    hipLaunchKernelGGL((k_m2p<T, PP, XB>), grid, block, lds, st, tl, n, nsplit, tabs.taps, tabs.m2p_off, lvs, Dst); \
    break;
    AFMM_M2P(1, 0) AFMM_M2P(2, 0) AFMM_M2P(3, 0) AFMM_M2P(4, 0) AFMM_M2P(5, 0) AFMM_M2P(6, 0) AFMM_M2P(7, 0)
    AFMM_M2P(8, 0) AFMM_M2P(1, 1) AFMM_M2P(2, 1) AFMM_M2P(3, 1) AFMM_M2P(4, 1) AFMM_M2P(5, 1) AFMM_M2P(6, 1)
    AFMM_M2P(7, 1)
#undef AFMM_M2P
    case 8 * 2 + 1:
      if constexpr (sizeof(T) == 4) {
        hipLaunchKernelGGL((k_m2p<T, 8, true>), grid, block, lds, st, tl, n, nsplit, tabs.taps, tabs.m2p_off, lvs, Dst);
        break;
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_m2p(int p, bool fp32, const MfmaTiles& mt, int t0, int n, int nsplit, int shape,
                      const MfmaTables& tabs, const LevelDev* lvs, const TablesDev<float>& t32,
                      const TablesDev<double>& t64, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (fp32) return m2p_dispatch<float>(p, mt, t0, n, nsplit, tabs, lvs, t32.Dstage, shape, st);
  return m2p_dispatch<double>(p, mt, t0, n, nsplit, tabs, lvs, t64.Dstage, shape, st);
}

int m2p_columns(int p, bool fp32) {
  (void)p;
  (void)fp32;
  return 16;
}

// Tile shapes of the M2P launch: 0 the direct form (16 groups per wave), 1 the
// row-staged form (16 groups), 2 the row-staged form with two tiles of one
// parity class per wave (32 groups; up to p = 5, where its registers fit),
// 3 the direct form with row-wise B loads passed over the crossbar (16
// groups).  The staged forms are instantiated for the FP32 kernels only.
bool m2p_shape_ok(int p, bool fp32, int shape) {
  if (shape == 0) return true;
  if (shape == 3) return fp32 || p <= 7;  // FP64 at p = 8 would spill
  if (!fp32) return false;
  return shape == 1 || (shape == 2 && p <= 5);
}
int m2p_shape_columns(int shape) { return shape == 2 ? 32 : 16; }

template <typename T>
static hipError_t m2l_dispatch(int p, const MfmaTiles& mt, int t0, int n, int nsplit, const MfmaTables& tabs,
                               const LevelDev* lvs, const T* Dst, hipStream_t st) {
  const int items = n * nsplit;
  const dim3 grid(8 * ((items + 7) / 8)), block(kBlock);
  const int32_t* tl = mt.tiles + (size_t)t0 * 17;
  switch (p) {
#define AFMM_M2L(PP)                                                                                          \
  case PP:                                                                                                    \
    hipLaunchKernelGGL((k_m2l_mfma<T, PP>), grid, block, 0, st, tl, n, nsplit, tabs.taps, tabs.m2l_off, lvs, \
                       Dst);                                                                                  \
    break;
    AFMM_M2L(1) AFMM_M2L(2) AFMM_M2L(3) AFMM_M2L(4) AFMM_M2L(5) AFMM_M2L(6) AFMM_M2L(7) AFMM_M2L(8)
#undef AFMM_M2L
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_m2l_taps(int p, bool fp32, const MfmaTiles& mt, int t0, int n, int nsplit, const MfmaTables& tabs,
                           const LevelDev* lvs, const TablesDev<float>& t32, const TablesDev<double>& t64,
                           hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (fp32) return m2l_dispatch<float>(p, mt, t0, n, nsplit, tabs, lvs, t32.Dstage, st);
  return m2l_dispatch<double>(p, mt, t0, n, nsplit, tabs, lvs, t64.Dstage, st);
}

template <typename T, typename TL>
static hipError_t l2l_dispatch(int p, const int32_t* grp, int ngrp, const TL* Lpar, const int32_t* rank0, T* Lout,
                               const T* Lpart, int nsplit, size_t stride, const T* w, const CommonDev& cm,
                               hipStream_t st) {
  const dim3 grid(ngrp), block(kBlock);
  if (nsplit < 1 || nsplit > 24) return hipErrorInvalidValue;
  const int ns = nsplit == 1 ? 0 : nsplit <= 8 ? 1 : 2;  // split bucket: 1, 8 or 24 partials
  switch (p * 3 + ns) {
#define AFMM_L2L(PP, NB, NSV)                                                                                    \
  case PP * 3 + NB:                                                                                              \
    hipLaunchKernelGGL((k_l2l<T, TL, PP, NSV>), grid, block, 0, st, grp, Lpar, rank0, Lout, Lpart, nsplit,       \
                       stride, w, cm.sumidx, cm.mi);                                                             \
    break;
#define AFMM_L2L3(PP) AFMM_L2L(PP, 0, 1) AFMM_L2L(PP, 1, 8) AFMM_L2L(PP, 2, 24)
    AFMM_L2L3(1) AFMM_L2L3(2) AFMM_L2L3(3) AFMM_L2L3(4) AFMM_L2L3(5) AFMM_L2L3(6) AFMM_L2L3(7) AFMM_L2L3(8)
#undef AFMM_L2L3
#undef AFMM_L2L
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_l2l(int p, bool fp32, bool parent_fp32, bool has_parent, int nsplit, const int32_t* grp, int ngrp,
                      const LevelDev& lv1, const LevelDev& lv0, const TablesDev<float>& t32,
                      const TablesDev<double>& t64, const CommonDev& cm, hipStream_t st) {
  if (ngrp == 0) return hipSuccess;
  const size_t stride = (size_t)lv0.nref * nmi(p);
  if (fp32) {
    if (parent_fp32)
      return l2l_dispatch<float, float>(p, grp, ngrp, has_parent ? lv1.L32 : nullptr, lv0.rank, lv0.L32,
                                        (const float*)lv0.Lpart, nsplit, stride, t32.l2lw, cm, st);
    return l2l_dispatch<float, double>(p, grp, ngrp, has_parent ? lv1.L64 : nullptr, lv0.rank, lv0.L32,
                                       (const float*)lv0.Lpart, nsplit, stride, t32.l2lw, cm, st);
  }
  return l2l_dispatch<double, double>(p, grp, ngrp, has_parent ? lv1.L64 : nullptr, lv0.rank, lv0.L64,
                                      (const double*)lv0.Lpart, nsplit, stride, t64.l2lw, cm, st);
}

template <typename T>
static hipError_t near_dispatch(int p, int ngrp, const int32_t* grp, const LevelDev& lv1, const LevelDev& lv0,
                                const TablesDev<T>& tb, const T* Lpar, const T* part, const T* nmp, double G,
                                double h, double cself, double* phi, double* acc, hipStream_t st) {
  const int ntiles = (ngrp + 15) / 16;
  const dim3 grid(8 * ((ntiles + 7) / 8)), block(kBlock);
  switch (p) {
#define AFMM_NEAR(PP)                                                                                         \
  case PP:                                                                                                    \
    hipLaunchKernelGGL((k_near<T, PP>), grid, block, 0, st, grp, ngrp, lv1, lv0, tb.nearA, Lpar, part, nmp,  \
                       G, h, cself, phi, acc);                                                                \
    break;
    AFMM_NEAR(1) AFMM_NEAR(2) AFMM_NEAR(3) AFMM_NEAR(4) AFMM_NEAR(5) AFMM_NEAR(6) AFMM_NEAR(7) AFMM_NEAR(8)
#undef AFMM_NEAR
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_near(int p, bool fp32, int l, int l_first, const int32_t* grp, int ngrp, const LevelDev& lv1,
                       const LevelDev& lv0, const LevelDev& lvp, const TablesDev<float>& t32,
                       const TablesDev<double>& t64, const CommonDev& cm, const void* part, const void* nmp,
                       double G, double h, double cself, double* phi, double* acc, hipStream_t st) {
  (void)cm;
  (void)lvp;
  if (ngrp == 0) return hipSuccess;
  const bool has_far = (l - 1) >= l_first;
  if (fp32)
    return near_dispatch<float>(p, ngrp, grp, lv1, lv0, t32, has_far ? lv1.L32 : nullptr, (const float*)part,
                                (const float*)nmp, G, h, cself, phi, acc, st);
  return near_dispatch<double>(p, ngrp, grp, lv1, lv0, t64, has_far ? lv1.L64 : nullptr, (const double*)part,
                               (const double*)nmp, G, h, cself, phi, acc, st);
}

template <typename T>
static hipError_t near_m2p_dispatch(int p, const int32_t* grp, int ngrp, const LevelDev& lv1, const LevelDev& lv0,
                                    const LevelDev& lvp, const T* Dsame, const T* S0, T* nmp, hipStream_t st) {
  const dim3 grid(ngrp), block(kBlock);
  switch (p) {
#define AFMM_NM2P(PP)                                                                                          \
  case PP:                                                                                                     \
    hipLaunchKernelGGL((k_near_m2p<T, PP>), grid, block, 0, st, grp, ngrp, lv1, lv0, lvp, Dsame, S0, nmp);     \
    break;
    AFMM_NM2P(1) AFMM_NM2P(2) AFMM_NM2P(3) AFMM_NM2P(4) AFMM_NM2P(5) AFMM_NM2P(6) AFMM_NM2P(7) AFMM_NM2P(8)
#undef AFMM_NM2P
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_near_m2p(int p, bool fp32, const int32_t* grp, int ngrp, const LevelDev& lv1, const LevelDev& lv0,
                           const LevelDev& lvp, const TablesDev<float>& t32, const TablesDev<double>& t64, void* nmp,
                           hipStream_t st) {
  if (ngrp == 0) return hipSuccess;
  if (fp32) return near_m2p_dispatch<float>(p, grp, ngrp, lv1, lv0, lvp, t32.Dsame, lv0.S32, (float*)nmp, st);
  return near_m2p_dispatch<double>(p, grp, ngrp, lv1, lv0, lvp, t64.Dsame, lv0.Sc64, (double*)nmp, st);
}

}  // namespace afmm
