// Periodic boxes: the far operator of FMM level 2 (host table and kernel).
//
// With AFMM_PERIODIC the box is a torus and the potential that of the masses
// with a uniform neutralising background, zero on average over the box (the
// Ewald sum).  Every neighbour row wraps around the box, so the levels >= 3
// already see the images of cells in the 3^3 block of boxes around the box.
// What they do not see reaches the local expansions of the 64 level-2 cells
// from all 64 level-2 cells s through one fixed operator per (octant of the
// target y, offset s - y):
//   T = Tlat(c_y - c_s) + sum over the block images n whose level-1 father
//       does not touch the target's level-1 ancestor of D(c_y - c_s - n L),
//   Tlat_g(d) = d^g(-F)(d),  F = Ewald sum of 1/r less its 27 nearest images,
// the second term being the level-1 interaction list of level 2 taken at
// level-2 resolution (M2L from level-1 sources would converge far slower).
// This extends the paper's isolated method (Sec. 5 names periodic domains as
// future work).
#include <hip/hip_runtime.h>

#include <array>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "afmm_internal.h"

namespace afmm {

namespace {

// Derivatives of a radial function h(|x|) at x for every multi-index of
// degree <= n (graded order), from q_m = ((1/rho) d/drho)^m h, m <= n:
// with R(m, 0) = q_m and R(m, g + e_i) = x_i R(m+1, g) + g_i R(m+1, g - e_i),
// d^g h = R(0, g).
void radial_derivs(int n, const long double x[3], const long double* q, long double* out) {
  const int K = nmi(n);
  std::vector<long double> R((size_t)(n + 1) * K, 0.0L);
  std::vector<int> g3(3 * K);
  for (int d = 0, idx = 0; d <= n; ++d)
    for (int a = d; a >= 0; --a)
      for (int b = d - a; b >= 0; --b, ++idx) {
        g3[3 * idx] = a;
        g3[3 * idx + 1] = b;
        g3[3 * idx + 2] = d - a - b;
      }
  for (int g = 0; g < K; ++g) {
    const int* gg = &g3[3 * g];
    const int deg = gg[0] + gg[1] + gg[2];
    for (int m = 0; m + deg <= n; ++m) {
      if (deg == 0) {
        R[(size_t)m * K] = q[m];
        continue;
      }
      const int i = gg[0] ? 0 : gg[1] ? 1 : 2;
      int lo[3] = {gg[0], gg[1], gg[2]};
      lo[i] -= 1;
      long double v = x[i] * R[(size_t)(m + 1) * K + mi_index(lo[0], lo[1], lo[2])];
      if (lo[i] > 0) {
        int lo2[3] = {lo[0], lo[1], lo[2]};
        lo2[i] -= 1;
        v += lo[i] * R[(size_t)(m + 1) * K + mi_index(lo2[0], lo2[1], lo2[2])];
      }
      R[(size_t)m * K + g] = v;
    }
  }
  for (int g = 0; g < K; ++g) out[g] = R[g];
}

// q_m of erfc(al rho)/rho (erf_part = false) or of -erf(al rho)/rho
// (erf_part = true), rho > 0:  ((1/rho) d/drho)^m erfc(al rho)/rho = (-1)^m B_m
// with B_0 = erfc(al rho)/rho and
// B_m = ((2m - 1) B_{m-1} + (2 al^2)^(m-1) 2 al/sqrt(pi) exp(-al^2 rho^2)) / rho^2,
// and ((1/rho) d/drho)^m 1/rho = (-1)^m (2m - 1)!! / rho^(2m + 1).
void radial_q(int n, long double rho, long double al, bool erf_part, long double* q) {
  const long double pi = 3.141592653589793238462643383279502884L;
  const long double r2 = rho * rho;
  long double B = std::erfc(al * rho) / rho;                       // B_m
  long double t = 2.0L * al / std::sqrt(pi) * std::exp(-al * al * r2);
  long double inv = 1.0L / rho, dfact = 1.0L;                        // 1/rho^(2m+1), (2m-1)!!
  for (int m = 0; m <= n; ++m) {
    if (m > 0) {
      B = ((2 * m - 1) * B + t) / r2;
      t *= 2.0L * al * al;
      inv /= r2;
      dfact *= (long double)(2 * m - 1);
    }
    const long double sg = (m & 1) ? -1.0L : 1.0L;
    q[m] = erf_part ? -sg * (dfact * inv - B) : sg * B;
  }
}

// Tlat_g(d) for |g| <= n on the unit box (Ewald split al = 1.8; images |n_i| <= 4
// and reciprocal vectors |m_i| <= 6 leave out terms below 1e-16 of the kept
// ones for |d_i| <= 3/4).  kpow[m][g] = k^g of reciprocal vector m, precomputed.
void lattice_tensor(int n, const long double d[3], const std::vector<std::array<long double, 3>>& kvec,
                    const std::vector<long double>& kw, const std::vector<long double>& kpow, long double* out) {
  const long double pi = 3.141592653589793238462643383279502884L, al = 1.8L;
  const int K = nmi(n);
  std::vector<long double> acc(K, 0.0L), t(K), q(n + 1);
  for (int a = -4; a <= 4; ++a)
    for (int b = -4; b <= 4; ++b)
      for (int c = -4; c <= 4; ++c) {
        const bool nearimg = a >= -1 && a <= 1 && b >= -1 && b <= 1 && c >= -1 && c <= 1;
        const long double x[3] = {d[0] + a, d[1] + b, d[2] + c};
        const long double rho = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        if (rho == 0.0L) {
          // -erf(al rho)/rho is a series in rho^2: q_m(0) = -2 al/sqrt(pi) (-2 al^2)^m / (2m + 1)
          long double pw = 1.0L;
          for (int m = 0; m <= n; ++m) {
            q[m] = -2.0L * al / std::sqrt(pi) * pw / (2 * m + 1);
            pw *= -2.0L * al * al;
          }
        } else {
          radial_q(n, rho, al, nearimg, q.data());
        }
        radial_derivs(n, x, q.data(), t.data());
        for (int g = 0; g < K; ++g) acc[g] += t[g];
      }
  // reciprocal part: d^g cos(k.r) = Re(i^|g| k^g exp(i k.r))
  for (size_t j = 0; j < kvec.size(); ++j) {
    const long double kd = kvec[j][0] * d[0] + kvec[j][1] * d[1] + kvec[j][2] * d[2];
    const long double cs = std::cos(kd), sn = std::sin(kd);
    const long double* kp = &kpow[j * K];
    int deg = 0;
    for (int g = 0; g < K; ++g) {
      while (nmi(deg) <= g) ++deg;  // deg = |g|
      const int r = deg & 3;
      const long double ph = r == 0 ? cs : r == 1 ? -sn : r == 2 ? -cs : sn;
      acc[g] += kw[j] * ph * kp[g];
    }
  }
  acc[0] -= pi / (al * al);
  for (int g = 0; g < K; ++g) out[g] = -acc[g];
}

// D_g = d^g(-1/r) at R for |g| <= n (radial derivatives of 1/r)
void coulomb_derivs(int n, const long double R[3], long double* out) {
  std::vector<long double> q(n + 1);
  const long double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
  long double v = -1.0L / std::sqrt(r2), dfact = 1.0L;
  for (int m = 0; m <= n; ++m) {
    if (m > 0) {
      dfact *= (long double)(2 * m - 1);
      v /= r2;
    }
    q[m] = ((m & 1) ? -1.0L : 1.0L) * dfact * v;   // ((1/rho) d/drho)^m (-1/rho)
  }
  radial_derivs(n, R, q.data(), out);
}

}  // namespace

// The level-2 far operator in level-2 units, [8 target octants][343 offsets][K]:
// element ((oy * 343 + di) * K + g) with di = (ex+3) + 7 (ey+3) + 49 (ez+3),
// e = s - y in level-2 cells, T~_g = (1/4)^(1+|g|) T_g on the unit box.
// Computed once per order and kept (shared by every periodic plan of that p).
std::shared_ptr<const std::vector<double>> periodic_far_table(int p) {
  static std::mutex mu;
  static std::map<int, std::shared_ptr<const std::vector<double>>> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(p);
  if (it != cache.end()) return it->second;
  const int K = nmi(p);
  const long double pi = 3.141592653589793238462643383279502884L, al = 1.8L;
  std::vector<std::array<long double, 3>> kvec;
  std::vector<long double> kw, kpow;
  for (int a = -6; a <= 6; ++a)
    for (int b = -6; b <= 6; ++b)
      for (int c = -6; c <= 6; ++c) {
        if (!a && !b && !c) continue;
        const std::array<long double, 3> k = {2 * pi * a, 2 * pi * b, 2 * pi * c};
        const long double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        kvec.push_back(k);
        kw.push_back(4.0L * pi * std::exp(-k2 / (4.0L * al * al)) / k2);
        for (int d = 0; d <= p; ++d)
          for (int x = d; x >= 0; --x)
            for (int y = d - x; y >= 0; --y) {
              long double v = 1.0L;
              for (int i = 0; i < x; ++i) v *= k[0];
              for (int i = 0; i < y; ++i) v *= k[1];
              for (int i = 0; i < d - x - y; ++i) v *= k[2];
              kpow.push_back(v);
            }
      }
  auto T = std::make_shared<std::vector<double>>((size_t)8 * kNumD * K, 0.0);
  std::vector<long double> scale(K);
  for (int g = 0, deg = 0; g < K; ++g) {
    while (nmi(deg) <= g) ++deg;      // deg = |g|
    scale[g] = std::pow(0.25L, deg + 1);
  }
  // the offsets are independent: each worker fills the rows of its own range
  parallel_ranges(kNumD, std::min(kNumD, host_threads()), [&](int64_t d0, int64_t d1, int) {
    std::vector<long double> lat(K), D(K);
    for (int di = (int)d0; di < (int)d1; ++di) {
      const int e[3] = {di % 7 - 3, (di / 7) % 7 - 3, di / 49 - 3};
      const long double R[3] = {-0.25L * e[0], -0.25L * e[1], -0.25L * e[2]};   // c_y - c_s
      lattice_tensor(p, R, kvec, kw, kpow, lat.data());
      for (int oy = 0; oy < 8; ++oy) {
        std::vector<long double> acc(lat);
        for (int n = 0; n < 27; ++n) {
          const int nn[3] = {n % 3 - 1, (n / 3) % 3 - 1, n / 9 - 1};
          // the image's level-1 father relative to the target's, per axis:
          // floor((o_y + e + 4 n) / 2); the image is far when one exceeds 1
          bool far = false;
          for (int i = 0; i < 3; ++i) {
            const int v = ((oy >> i) & 1) + e[i] + 4 * nn[i];
            const int f1 = v >= 0 ? v / 2 : -((1 - v) / 2);
            far = far || f1 < -1 || f1 > 1;
          }
          if (!far) continue;
          const long double Rn[3] = {R[0] - nn[0], R[1] - nn[1], R[2] - nn[2]};
          coulomb_derivs(p, Rn, D.data());
          for (int g = 0; g < K; ++g) acc[g] += D[g];
        }
        double* row = &(*T)[((size_t)oy * kNumD + di) * K];
        for (int g = 0; g < K; ++g) row[g] = (double)(acc[g] * scale[g]);
      }
    }
  });
  cache[p] = T;
  return T;
}

// L~(y) = sum_s sum_a cf_a T~[o_y][s - y]_{a+b} S~_a(s) for the 64 level-2
// cells of each hierarchy (all refined: level 2 lies above levelmin, so rank =
// cell index; hierarchy j of a batch owns cells 64 j .. 64 j + 63, and local
// cell c = 8 o1 + o2 sits at 2 bit(o1) + bit(o2) per axis).  Block (target,
// hierarchy), the hierarchy's 64 source rows in LDS, thread = coefficient b.
template <int P>
__global__ __launch_bounds__(256) void k_periodic_far(LevelDev lv2, const double* __restrict__ T,
                                                      const double* __restrict__ cf,
                                                      const int16_t* __restrict__ sumidx,
                                                      const int8_t* __restrict__ mi) {
  constexpr int K = nmi(P);
  __shared__ double sS[64 * K];
  const int y = blockIdx.x;
  const size_t base = (size_t)blockIdx.y * 64;   // the hierarchy's first level-2 cell
  for (int i = threadIdx.x; i < 64 * K; i += 256) sS[i] = cf[i % K] * lv2.S64[base * K + i];
  __syncthreads();
  const int b = threadIdx.x;
  if (b >= K) return;
  auto axis = [](int c, int i) { return 2 * ((c >> (3 + i)) & 1) + ((c >> i) & 1); };
  const int y0 = axis(y, 0), y1 = axis(y, 1), y2 = axis(y, 2), oy = y & 7;
  const int na = nmi(P - mi[4 * b + 3]);
  const int16_t* si = sumidx + (size_t)b * K;
  double acc = 0.0;
  for (int s = 0; s < 64; ++s) {
    const int di = (axis(s, 0) - y0 + 3) + 7 * (axis(s, 1) - y1 + 3) + 49 * (axis(s, 2) - y2 + 3);
    const double* Tr = T + ((size_t)oy * kNumD + di) * K;
    const double* Sr = sS + s * K;
    for (int a = 0; a < na; ++a) acc += Tr[si[a]] * Sr[a];
  }
  if (lv2.L64) lv2.L64[(base + y) * K + b] = acc;
  else lv2.L32[(base + y) * K + b] = (float)acc;
}

// Adjoint: the bars of the level-2 multipoles, S~bar_a(s) += cf_a sum_y sum_b
// T~[o_y][s - y]_{a+b} L~bar_b(y) (after the source-copy bars of level 2 became
// multipole bars).  One block per source, the 64 L~bar rows in LDS, thread =
// coefficient a.
template <int P>
__global__ __launch_bounds__(256) void k_adj_periodic_far(LevelDev lv2, const double* __restrict__ T,
                                                          const double* __restrict__ cf,
                                                          const int16_t* __restrict__ sumidx,
                                                          const int8_t* __restrict__ mi) {
  constexpr int K = nmi(P);
  __shared__ double sL[64 * K];
  const int s = blockIdx.x;
  for (int i = threadIdx.x; i < 64 * K; i += 256) sL[i] = lv2.lbar[i];
  __syncthreads();
  const int a = threadIdx.x;
  if (a >= K) return;
  auto axis = [](int c, int i) { return 2 * ((c >> (3 + i)) & 1) + ((c >> i) & 1); };
  const int s0 = axis(s, 0), s1 = axis(s, 1), s2 = axis(s, 2);
  const int nb = nmi(P - mi[4 * a + 3]);
  const int16_t* si = sumidx + (size_t)a * K;   // index of a + b
  double acc = 0.0;
  for (int y = 0; y < 64; ++y) {
    const int di = (s0 - axis(y, 0) + 3) + 7 * (s1 - axis(y, 1) + 3) + 49 * (s2 - axis(y, 2) + 3);
    const double* Tr = T + ((size_t)(y & 7) * kNumD + di) * K;
    const double* Lr = sL + y * K;
    for (int b = 0; b < nb; ++b) acc += Tr[si[b]] * Lr[b];
  }
  lv2.sbar[(size_t)s * K + a] += cf[a] * acc;
}

hipError_t launch_adj_periodic_far(int p, const LevelDev& lv2, const double* T, const double* cf,
                                   const CommonDev& cm, hipStream_t st) {
  if (lv2.nref != 64 || !lv2.lbar || !lv2.sbar || !T || !cf) return hipErrorInvalidValue;
  switch (p) {
#define X(PP)                                                                                              \
  case PP:                                                                                                 \
    hipLaunchKernelGGL((k_adj_periodic_far<PP>), dim3(64), dim3(256), 0, st, lv2, T, cf, cm.sumidx, cm.mi); \
    break;
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_periodic_far(int p, const LevelDev& lv2, const double* T, const double* cf, const CommonDev& cm,
                               hipStream_t st) {
  if (lv2.nref <= 0 || lv2.nref % 64 || !lv2.S64 || (!lv2.L64 && !lv2.L32) || !T || !cf)
    return hipErrorInvalidValue;
  const dim3 grid(64, lv2.nref / 64);
  switch (p) {
#define X(PP)                                                                                          \
  case PP:                                                                                             \
    hipLaunchKernelGGL((k_periodic_far<PP>), grid, dim3(256), 0, st, lv2, T, cf, cm.sumidx, cm.mi);     \
    break;
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace afmm
