// Particle-mesh coupling of the solver for time loops (Sec. 1: particle masses
// are deposited onto the AMR cells by cloud-in-cell; Sec. 4: the binary-orbit
// test, two point masses advanced by a fixed-step leapfrog on an AMR grid
// that keeps them on the finest level).
//
//   host:   a graded hierarchy refined around the particles' clouds
//           (afmm_particle_hierarchy_*), rebuilt by the caller whenever the
//           particles have moved;
//   device: CIC deposition of particle masses onto the leaf cells of one level,
//           CIC interpolation of the cell accelerations / potentials back to
//           the particles, leapfrog kick and drift.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "afmm_internal.h"

namespace afmm {
afmm_status pm_fail(afmm_status s, const char* msg);
// Morton keys (x in the lowest bit of each triple) of the cells of level l of a
// plan, in the plan's cell order (ascending), uploaded on first use; n_out the
// level's cell count.  Defined with the plan (afmm_host.hip).
afmm_status plan_level_keys(afmm_plan* P, int level, const uint64_t** keys, const LevelDev** lv);
}  // namespace afmm

using namespace afmm;

// ---------------------------------------------------------------------------
// host: hierarchy refined around particles

namespace {

inline uint64_t key3(int64_t i, int64_t j, int64_t k, int l) {
  return ((uint64_t)i << (2 * l)) | ((uint64_t)j << l) | (uint64_t)k;
}
inline void unkey3(uint64_t key, int l, int64_t* c) {
  const uint64_t m = ((uint64_t)1 << l) - 1;
  c[0] = (int64_t)(key >> (2 * l));
  c[1] = (int64_t)((key >> l) & m);
  c[2] = (int64_t)(key & m);
}

}  // namespace

struct afmm_particle_hierarchy {
  int32_t levelmin = 0, levelmax = 0;
  std::vector<int64_t> ncell;
  std::vector<int32_t> ijk;
  std::vector<uint8_t> refined;
};

// Refine, at every level l < levelmax, the cells within `nexpand` cells
// (Chebyshev distance, clipped to the box) of the 2x2x2 cloud of a particle at
// level l; then close the strong grading rule (a refined level-l cell needs the
// 27 level-(l-1) neighbours of its father refined) bottom-up, and repeat both
// to a fixed point (each step only adds refinement).  Cells appear level by
// level, each level in Morton order.
static afmm_status particle_hierarchy_impl(int32_t levelmin, int32_t levelmax, int32_t nexpand, int64_t np,
                                           const double* pos, double boxlen, afmm_particle_hierarchy** out) {
  if (!out || (np > 0 && !pos)) return pm_fail(AFMM_E_INVALID_ARG, "null argument");
  *out = nullptr;
  if (levelmin < 1 || levelmax < levelmin || levelmax > 20)
    return pm_fail(AFMM_E_INVALID_ARG, "levels must satisfy 1 <= levelmin <= levelmax <= 20");
  if (nexpand < 0 || np < 0 || !(boxlen > 0)) return pm_fail(AFMM_E_INVALID_ARG, "bad nexpand, count or boxlen");
  for (int64_t p = 0; p < 3 * np; ++p)
    if (!std::isfinite(pos[p]) || pos[p] < 0 || pos[p] >= boxlen)
      return pm_fail(AFMM_E_INVALID_ARG, "particle outside the box");
  const int nl = levelmax - levelmin;  // refinable levels
  // wanted refinement per level, from the particles
  std::vector<std::vector<uint64_t>> want(nl);
  for (int i = 0; i < nl; ++i) {
    const int l = levelmin + i;
    const int64_t n = (int64_t)1 << l;
    const double inv_h = (double)n / boxlen;
    auto& w = want[i];
    for (int64_t p = 0; p < np; ++p) {
      int64_t lo[3], hi[3];
      for (int d = 0; d < 3; ++d) {
        const int64_t c0 = (int64_t)std::floor(pos[3 * p + d] * inv_h - 0.5);  // cloud cells c0, c0 + 1
        lo[d] = std::max<int64_t>(0, c0 - nexpand);
        hi[d] = std::min<int64_t>(n - 1, c0 + 1 + nexpand);
      }
      for (int64_t a = lo[0]; a <= hi[0]; ++a)
        for (int64_t b = lo[1]; b <= hi[1]; ++b)
          for (int64_t c = lo[2]; c <= hi[2]; ++c) w.push_back(key3(a, b, c, l));
    }
    std::sort(w.begin(), w.end());
    w.erase(std::unique(w.begin(), w.end()), w.end());
  }
  std::vector<std::vector<uint64_t>> R(nl);  // refined keys per level (sorted)
  auto exists_children = [&](const std::vector<uint64_t>& ref, int l) {
    std::vector<uint64_t> ch;
    ch.reserve(ref.size() * 8);
    for (uint64_t k : ref) {
      int64_t c[3];
      unkey3(k, l, c);
      for (int o = 0; o < 8; ++o) ch.push_back(key3(2 * c[0] + (o & 1), 2 * c[1] + ((o >> 1) & 1), 2 * c[2] + ((o >> 2) & 1), l + 1));
    }
    std::sort(ch.begin(), ch.end());
    return ch;
  };
  for (int it = 0; it < 64; ++it) {
    bool changed = false;
    // top-down: wanted cells that exist (level levelmin is complete and the
    // wanted keys are clipped to the box, so there every wanted cell exists)
    std::vector<uint64_t> cells;  // cells of level l > levelmin (sorted)
    for (int i = 0; i < nl; ++i) {
      const int l = levelmin + i;
      std::vector<uint64_t> merged;
      if (i == 0) {
        std::set_union(R[0].begin(), R[0].end(), want[0].begin(), want[0].end(), std::back_inserter(merged));
      } else {
        std::vector<uint64_t> add;
        std::set_intersection(want[i].begin(), want[i].end(), cells.begin(), cells.end(), std::back_inserter(add));
        std::vector<uint64_t> u;
        std::set_union(R[i].begin(), R[i].end(), add.begin(), add.end(), std::back_inserter(u));
        // refined cells must exist
        std::set_intersection(u.begin(), u.end(), cells.begin(), cells.end(), std::back_inserter(merged));
      }
      if (merged.size() != R[i].size()) changed = true;
      R[i].swap(merged);
      cells = exists_children(R[i], l);
    }
    // bottom-up grading closure
    for (int i = nl - 1; i >= 1; --i) {
      const int l = levelmin + i;
      if (R[i].empty()) continue;
      std::vector<uint64_t> need;
      const int64_t np1 = (int64_t)1 << (l - 1);
      for (uint64_t k : R[i]) {
        int64_t c[3];
        unkey3(k, l, c);
        for (int e = 0; e < 27; ++e) {
          const int64_t q[3] = {(c[0] >> 1) + e % 3 - 1, (c[1] >> 1) + (e / 3) % 3 - 1, (c[2] >> 1) + e / 9 - 1};
          if (q[0] < 0 || q[0] >= np1 || q[1] < 0 || q[1] >= np1 || q[2] < 0 || q[2] >= np1) continue;
          need.push_back(key3(q[0], q[1], q[2], l - 1));
        }
      }
      std::sort(need.begin(), need.end());
      need.erase(std::unique(need.begin(), need.end()), need.end());
      std::vector<uint64_t> merged;
      std::set_union(R[i - 1].begin(), R[i - 1].end(), need.begin(), need.end(), std::back_inserter(merged));
      if (merged.size() != R[i - 1].size()) changed = true;
      R[i - 1].swap(merged);
    }
    if (!changed) break;
    if (it == 63) return pm_fail(AFMM_E_INVALID_ARG, "refinement did not reach a fixed point");
  }
  std::unique_ptr<afmm_particle_hierarchy> H(new afmm_particle_hierarchy());
  H->levelmin = levelmin;
  // every level in Morton order (the order the plan keeps its levels in, so
  // that a plan built from this hierarchy need not sort it)
  auto emit = [&](const std::vector<uint64_t>& cells, int l, const std::vector<uint64_t>& ref) {
    const int64_t n = (int64_t)cells.size();
    std::vector<std::pair<uint64_t, uint64_t>> mk((size_t)n);  // (Morton key, (i, j, k)-major key)
    parallel_ranges(n, parts_for(n), [&](int64_t b, int64_t e, int) {
      for (int64_t i = b; i < e; ++i) {
        int64_t c[3];
        unkey3(cells[(size_t)i], l, c);
        mk[(size_t)i] = {morton3((uint32_t)c[0], (uint32_t)c[1], (uint32_t)c[2]), cells[(size_t)i]};
      }
    });
    std::sort(mk.begin(), mk.end());
    const size_t b0 = H->refined.size();
    H->ncell.push_back(n);
    H->ijk.resize(3 * (b0 + (size_t)n));
    H->refined.resize(b0 + (size_t)n);
    int32_t* ijk = H->ijk.data() + 3 * b0;
    uint8_t* on = H->refined.data() + b0;
    parallel_ranges(n, parts_for(n), [&](int64_t b, int64_t e, int) {
      for (int64_t i = b; i < e; ++i) {
        const uint64_t k = mk[(size_t)i].second;
        int64_t c[3];
        unkey3(k, l, c);
        ijk[3 * i] = (int32_t)c[0];
        ijk[3 * i + 1] = (int32_t)c[1];
        ijk[3 * i + 2] = (int32_t)c[2];
        on[i] = std::binary_search(ref.begin(), ref.end(), k) ? 1 : 0;
      }
    });
  };
  const std::vector<uint64_t> none;
  {
    // level levelmin: the whole grid; a complete grid's Morton keys are 0 .. n - 1
    const int64_t n0 = (int64_t)1 << levelmin, nb = n0 * n0 * n0;
    const std::vector<uint64_t>& ref = nl > 0 ? R[0] : none;
    size_t total = (size_t)nb;
    for (int i = 0; i < nl; ++i) total += 8 * R[i].size();
    H->ijk.reserve(3 * total);
    H->refined.reserve(total);
    std::vector<uint8_t> flag((size_t)nb, 0);  // by (i, j, k)-major key
    for (uint64_t k : ref) flag[(size_t)k] = 1;
    H->ijk.resize(3 * (size_t)nb);
    H->refined.resize((size_t)nb);
    H->ncell.push_back(nb);
    int32_t* ijk = H->ijk.data();
    uint8_t* on = H->refined.data();
    parallel_ranges(nb, parts_for(nb), [&](int64_t b, int64_t e, int) {
      for (int64_t m = b; m < e; ++m) {
        uint32_t c[3] = {0, 0, 0};
        for (int bit = 0; bit < levelmin; ++bit)
          for (int d = 0; d < 3; ++d) c[d] |= (uint32_t)((m >> (3 * bit + d)) & 1) << bit;
        ijk[3 * m] = (int32_t)c[0];
        ijk[3 * m + 1] = (int32_t)c[1];
        ijk[3 * m + 2] = (int32_t)c[2];
        on[m] = flag[(size_t)key3(c[0], c[1], c[2], levelmin)];
      }
    });
  }
  std::vector<uint64_t> cells = nl > 0 ? exists_children(R[0], levelmin) : std::vector<uint64_t>();
  int top = levelmin;
  for (int l = levelmin + 1; l <= levelmax && !cells.empty(); ++l) {
    top = l;
    const std::vector<uint64_t>& ref = l < levelmax ? R[l - levelmin] : none;
    emit(cells, l, ref);
    if (l < levelmax) cells = exists_children(ref, l);
  }
  H->levelmax = top;
  *out = H.release();
  return AFMM_OK;
}

extern "C" afmm_status afmm_particle_hierarchy_create(int32_t levelmin, int32_t levelmax, int32_t nexpand, int64_t np,
                                                     const double* pos, double boxlen,
                                                     afmm_particle_hierarchy** out) {
  try {
    return particle_hierarchy_impl(levelmin, levelmax, nexpand, np, pos, boxlen, out);
  } catch (const std::bad_alloc&) {
    return pm_fail(AFMM_E_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return pm_fail(AFMM_E_INVALID_ARG, "internal error");
  }
}

extern "C" afmm_status afmm_particle_hierarchy_view(const afmm_particle_hierarchy* H, afmm_hierarchy* out) {
  if (!H || !out) return pm_fail(AFMM_E_INVALID_ARG, "null argument");
  out->levelmin = H->levelmin;
  out->levelmax = H->levelmax;
  out->ncell = H->ncell.data();
  out->ijk = H->ijk.data();
  out->refined = H->refined.data();
  return AFMM_OK;
}

extern "C" afmm_status afmm_particle_hierarchy_destroy(afmm_particle_hierarchy* H) {
  delete H;
  return AFMM_OK;
}

// ---------------------------------------------------------------------------
// device: CIC deposition / interpolation, leapfrog

namespace {

__device__ inline uint64_t spread3(uint64_t v) {
  v &= 0x1fffff;
  v = (v | v << 32) & 0x1f00000000ffffULL;
  v = (v | v << 16) & 0x1f0000ff0000ffULL;
  v = (v | v << 8) & 0x100f00f00f00f00fULL;
  v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
  v = (v | v << 2) & 0x1249249249249249ULL;
  return v;
}

// Leaf slot of cell (i, j, k) at the level whose sorted Morton keys are
// keys[0..n), or -1 if the cell is absent or refined.
__device__ inline int leaf_slot(int64_t i, int64_t j, int64_t k, const uint64_t* __restrict__ keys, int n,
                                const int32_t* __restrict__ rank, const int32_t* __restrict__ slot) {
  const uint64_t key = spread3((uint64_t)i) | (spread3((uint64_t)j) << 1) | (spread3((uint64_t)k) << 2);
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (keys[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  if (lo >= n || keys[lo] != key || rank[lo] >= 0) return -1;
  return slot[lo];
}

// the 8 cloud cells of a particle (cell indices and weights), or false if the
// cloud leaves the box
__device__ inline bool cloud(const double* x, double inv_h, int64_t nside, int64_t* c0, double* f) {
  for (int d = 0; d < 3; ++d) {
    const double u = x[d] * inv_h - 0.5;
    const double fl = floor(u);
    c0[d] = (int64_t)fl;
    f[d] = u - fl;
    if (c0[d] < 0 || c0[d] + 1 >= nside) return false;
  }
  return true;
}

}  // namespace

__global__ void k_fill(int64_t n, double* __restrict__ p) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

__global__ void k_cic_deposit(int64_t np, const double* __restrict__ pos, const double* __restrict__ m, double inv_h,
                              int64_t nside, const uint64_t* __restrict__ keys, int n,
                              const int32_t* __restrict__ rank, const int32_t* __restrict__ slot,
                              double* __restrict__ cell_mass, int* __restrict__ flag) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= np) return;
  int64_t c0[3];
  double f[3];
  if (!cloud(pos + 3 * p, inv_h, nside, c0, f)) {
    flag[0] = 1;
    return;
  }
  const double mp = m[p];
  for (int o = 0; o < 8; ++o) {
    const int ox = o & 1, oy = (o >> 1) & 1, oz = (o >> 2) & 1;
    const int s = leaf_slot(c0[0] + ox, c0[1] + oy, c0[2] + oz, keys, n, rank, slot);
    if (s < 0) {
      flag[0] = 1;
      continue;
    }
    const double w = (ox ? f[0] : 1.0 - f[0]) * (oy ? f[1] : 1.0 - f[1]) * (oz ? f[2] : 1.0 - f[2]);
    atomicAdd(cell_mass + s, w * mp);
  }
}

__global__ void k_cic_interp(int64_t np, const double* __restrict__ pos, double inv_h, int64_t nside,
                             const uint64_t* __restrict__ keys, int n, const int32_t* __restrict__ rank,
                             const int32_t* __restrict__ slot, const double* __restrict__ cell_acc,
                             const double* __restrict__ cell_phi, double* __restrict__ acc, double* __restrict__ phi,
                             int* __restrict__ flag) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= np) return;
  int64_t c0[3];
  double f[3];
  double a[3] = {0.0, 0.0, 0.0}, ph = 0.0;
  if (!cloud(pos + 3 * p, inv_h, nside, c0, f)) {
    flag[0] = 1;
  } else {
    for (int o = 0; o < 8; ++o) {
      const int ox = o & 1, oy = (o >> 1) & 1, oz = (o >> 2) & 1;
      const int s = leaf_slot(c0[0] + ox, c0[1] + oy, c0[2] + oz, keys, n, rank, slot);
      if (s < 0) {
        flag[0] = 1;
        continue;
      }
      const double w = (ox ? f[0] : 1.0 - f[0]) * (oy ? f[1] : 1.0 - f[1]) * (oz ? f[2] : 1.0 - f[2]);
      for (int d = 0; d < 3; ++d) a[d] += w * cell_acc[3 * (int64_t)s + d];
      if (cell_phi) ph += w * cell_phi[s];
    }
  }
  for (int d = 0; d < 3; ++d) acc[3 * p + d] = a[d];
  if (phi) phi[p] = ph;
}

__global__ void k_axpy3(int64_t n3, double dt, const double* __restrict__ x, double* __restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n3) y[i] += dt * x[i];
}
__global__ void k_flag_zero(int* __restrict__ flag) { flag[0] = 0; }

// ---------------------------------------------------------------------------
// entry points

namespace afmm {
afmm_status plan_pm_flag(afmm_plan* P, int** d_flag, int** h_flag);
double plan_boxlen(const afmm_plan* P);
}  // namespace afmm

static afmm_status pm_common(afmm_plan* P, int32_t level, int64_t np, const double* d_pos, const uint64_t** keys,
                             const LevelDev** lv, double* inv_h, int64_t* nside) {
  if (!P || np < 0 || (np > 0 && !d_pos)) return pm_fail(AFMM_E_INVALID_ARG, "null argument or negative count");
  afmm_status s = plan_level_keys(P, level, keys, lv);
  if (s) return s;
  *nside = (int64_t)1 << level;
  *inv_h = (double)*nside / plan_boxlen(P);
  return AFMM_OK;
}

static afmm_status pm_check_flag(afmm_plan* P, hipStream_t st, const char* what) {
  int *d_flag, *h_flag;
  afmm_status s = plan_pm_flag(P, &d_flag, &h_flag);
  if (s) return s;
  if (hipMemcpyAsync(h_flag, d_flag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return pm_fail(AFMM_E_DEVICE, "particle flag read back failed");
  if (*h_flag) return pm_fail(AFMM_E_INVALID_ARG, what);
  return AFMM_OK;
}

extern "C" afmm_status afmm_cic_deposit(afmm_plan* P, int32_t level, int64_t np, const double* d_pos,
                                        const double* d_pmass, double* d_cell_mass, void* hip_stream) {
  try {
    const uint64_t* keys;
    const LevelDev* lv;
    double inv_h;
    int64_t nside;
    afmm_status s = pm_common(P, level, np, d_pos, &keys, &lv, &inv_h, &nside);
    if (s) return s;
    if (!d_cell_mass || (np > 0 && !d_pmass)) return pm_fail(AFMM_E_INVALID_ARG, "null argument");
    afmm_plan_info info;
    if ((s = afmm_plan_get_info(P, &info))) return s;
    hipStream_t st = (hipStream_t)hip_stream;
    int *d_flag, *h_flag;
    if ((s = plan_pm_flag(P, &d_flag, &h_flag))) return s;
    hipLaunchKernelGGL(k_flag_zero, dim3(1), dim3(1), 0, st, d_flag);
    hipLaunchKernelGGL(k_fill, dim3((unsigned)std::min<int64_t>((info.ncell + 255) / 256, 4096)), dim3(256), 0, st,
                       (int64_t)info.ncell, d_cell_mass);
    if (np > 0)
      hipLaunchKernelGGL(k_cic_deposit, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, np, d_pos, d_pmass,
                         inv_h, nside, keys, lv->n, lv->rank, lv->slot, d_cell_mass, d_flag);
    if (hipGetLastError() != hipSuccess) return pm_fail(AFMM_E_DEVICE, "deposit launch failed");
    return pm_check_flag(P, st, "a particle cloud leaves the box or covers a cell that is not a leaf of the level");
  } catch (...) {
    return pm_fail(AFMM_E_OUT_OF_MEMORY, "host allocation failed");
  }
}

extern "C" afmm_status afmm_cic_interpolate(afmm_plan* P, int32_t level, int64_t np, const double* d_pos,
                                            const double* d_cell_acc, const double* d_cell_phi, double* d_acc,
                                            double* d_phi, void* hip_stream) {
  try {
    const uint64_t* keys;
    const LevelDev* lv;
    double inv_h;
    int64_t nside;
    afmm_status s = pm_common(P, level, np, d_pos, &keys, &lv, &inv_h, &nside);
    if (s) return s;
    if (np > 0 && (!d_cell_acc || !d_acc)) return pm_fail(AFMM_E_INVALID_ARG, "null argument");
    hipStream_t st = (hipStream_t)hip_stream;
    int *d_flag, *h_flag;
    if ((s = plan_pm_flag(P, &d_flag, &h_flag))) return s;
    hipLaunchKernelGGL(k_flag_zero, dim3(1), dim3(1), 0, st, d_flag);
    if (np > 0)
      hipLaunchKernelGGL(k_cic_interp, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, np, d_pos, inv_h, nside,
                         keys, lv->n, lv->rank, lv->slot, d_cell_acc, d_cell_phi, d_acc, d_phi, d_flag);
    if (hipGetLastError() != hipSuccess) return pm_fail(AFMM_E_DEVICE, "interpolation launch failed");
    return pm_check_flag(P, st, "a particle cloud leaves the box or covers a cell that is not a leaf of the level");
  } catch (...) {
    return pm_fail(AFMM_E_OUT_OF_MEMORY, "host allocation failed");
  }
}

extern "C" afmm_status afmm_particles_update(int64_t n3, double dt, const double* d_rate, double* d_state,
                                             void* hip_stream) {
  if (n3 < 0 || (n3 > 0 && (!d_rate || !d_state))) return pm_fail(AFMM_E_INVALID_ARG, "null argument");
  if (n3 == 0) return AFMM_OK;
  hipLaunchKernelGGL(k_axpy3, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, (hipStream_t)hip_stream, n3, dt,
                     d_rate, d_state);
  return hipGetLastError() == hipSuccess ? AFMM_OK : pm_fail(AFMM_E_DEVICE, "update launch failed");
}
