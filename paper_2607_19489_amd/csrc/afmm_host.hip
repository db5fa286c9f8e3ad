// Host runtime of the adaptive FMM: hierarchy validation, per-level Morton
// ordering, neighbour tables, group lists (the merged topology shared by all
// per-level trees, Sec. 3.1), translation tables, device memory, and the
// solve driver (Alg. 1-4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "afmm_internal.h"

namespace afmm {

thread_local std::string g_last_error;

static afmm_status fail(afmm_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

// Host containers may throw (std::bad_alloc on huge plans); no exception may
// cross the C ABI, so every entry point that allocates runs through this.
template <typename F>
static afmm_status guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(AFMM_E_OUT_OF_MEMORY, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(AFMM_E_INVALID_ARG, std::string("internal error: ") + e.what());
  } catch (...) {
    return fail(AFMM_E_INVALID_ARG, "internal error");
  }
}

// ---------------------------------------------------------------------------
// topology (host)

struct HostLevel {
  std::vector<int32_t> rank;     // [n]
  std::vector<int32_t> slot;     // [n]
  std::vector<int32_t> refcell;  // [nref]
  std::vector<int32_t> nbr;      // [nref * 27]
  int32_t n() const { return (int32_t)rank.size(); }
  int32_t nref() const { return (int32_t)refcell.size(); }
};

struct Topology {
  bool periodic = false;         // neighbour rows wrap around the box (AFMM_PERIODIC)
  int lmax = 0;                  // deepest level present
  int lmin_all = 1 << 30;        // smallest levelmin over hierarchies
  HostLevel lv[kMaxLevel];
  int64_t nslots = 0;
  std::vector<int32_t> leafgrp[kMaxLevel];  // index l: refined ranks at l-1 with a leaf child
  std::vector<int32_t> m2lgrp[kMaxLevel];   // index f: refined ranks at f-1 with a refined child
  std::vector<int32_t> nmgrp[kMaxLevel];    // index l: leafgrp entries with a refined level-l near candidate
  std::vector<int32_t> adjvgrp[kMaxLevel];  // index l: leafgrp entries with a coarse leaf neighbour or a
                                            // refined near candidate (adjoint VALU near relations)
  std::vector<int32_t> upleaf[kMaxLevel];   // index f: refined ranks at f whose 8 children are leaves
  std::vector<int32_t> upmix[kMaxLevel];    // index f: refined ranks at f with a refined child
  // per hierarchy
  std::vector<int32_t> levelmin, levelmax;
  std::vector<int64_t> slot_base, slot_count;
  std::vector<std::vector<int64_t>> level_off;  // flat slot offset of each AMR level (per hierarchy)
};

// LSD radix sort of (Morton key, caller index) pairs by key, 8 key bits per
// pass over the `bits` low bits that the keys use.  Each pass counts the
// digits of every range, then each range scatters its items after those of
// the same digit in earlier ranges: stable, so with distinct keys the order
// is that of std::sort, whatever the number of ranges.
static void radix_sort_keys(std::vector<std::pair<uint64_t, int32_t>>& v, int bits) {
  const int64_t n = (int64_t)v.size();
  const int parts = parts_for(n, 1 << 15);
  std::vector<std::pair<uint64_t, int32_t>> tmp(v.size());
  std::vector<std::array<size_t, 256>> cnt((size_t)parts);
  for (int shift = 0; shift < bits; shift += 8) {
    parallel_ranges(n, parts, [&](int64_t b, int64_t e, int t) {
      auto& c = cnt[(size_t)t];
      c.fill(0);
      for (int64_t i = b; i < e; ++i) ++c[(v[(size_t)i].first >> shift) & 255];
    });
    size_t run = 0;
    for (int d = 0; d < 256; ++d)
      for (int t = 0; t < parts; ++t) {
        const size_t k = cnt[(size_t)t][d];
        cnt[(size_t)t][d] = run;
        run += k;
      }
    parallel_ranges(n, parts, [&](int64_t b, int64_t e, int t) {
      auto& c = cnt[(size_t)t];
      for (int64_t i = b; i < e; ++i) tmp[c[(v[(size_t)i].first >> shift) & 255]++] = v[(size_t)i];
    });
    v.swap(tmp);
  }
}

// Append one hierarchy to the topology (levels 0..levelmax); slots are the
// hierarchy's flat cell indices offset by slot_base.
static afmm_status append_hierarchy(Topology& T, const afmm_hierarchy& h, int64_t slot_base) {
  if (!h.ncell || !h.ijk || !h.refined) return fail(AFMM_E_INVALID_ARG, "null hierarchy array");
  const int lmin = h.levelmin, lmax = h.levelmax;
  if (lmin < 1 || lmax < lmin || lmax > 20)
    return fail(AFMM_E_INVALID_ARG, "levels must satisfy 1 <= levelmin <= levelmax <= 20");
  const int nl = lmax - lmin + 1;
  std::vector<int64_t> off(nl + 1, 0);
  for (int i = 0; i < nl; ++i) {
    if (h.ncell[i] < 0) return fail(AFMM_E_INVALID_ARG, "negative cell count");
    off[i + 1] = off[i] + h.ncell[i];
  }
  if (h.ncell[0] != (int64_t)1 << (3 * lmin))
    return fail(AFMM_E_INCOMPLETE_OCT, "levelmin must be complete (8^levelmin cells)");
  if (T.periodic && lmin < 3) return fail(AFMM_E_UNSUPPORTED, "periodic boxes need levelmin >= 3");
  if (slot_base + off[nl] >= ((int64_t)1 << 31)) return fail(AFMM_E_INVALID_ARG, "more than 2^31 cells");

  // caller cells of each AMR level sorted by Morton key
  std::vector<std::vector<std::pair<uint64_t, int32_t>>> sorted(nl);
  for (int i = 0; i < nl; ++i) {
    const int l = lmin + i;
    const int64_t side = (int64_t)1 << l;
    auto& v = sorted[i];
    v.resize(h.ncell[i]);
    const int parts = parts_for(h.ncell[i], 4096);
    std::vector<int64_t> bad((size_t)parts, -1);  // first cell out of range in each range
    parallel_ranges(h.ncell[i], parts, [&](int64_t cb, int64_t ce, int part) {
      for (int64_t c = cb; c < ce; ++c) {
        const int32_t* x = h.ijk + 3 * (off[i] + c);
        if (x[0] < 0 || x[0] >= side || x[1] < 0 || x[1] >= side || x[2] < 0 || x[2] >= side) {
          bad[(size_t)part] = c;
          return;
        }
        v[(size_t)c] = {morton3(x[0], x[1], x[2]), (int32_t)c};
      }
    });
    for (int64_t c : bad)
      if (c >= 0) {
        char b[128];
        snprintf(b, sizeof b, "cell %lld of level %d out of range", (long long)c, l);
        return fail(AFMM_E_INVALID_ARG, b);
      }
    if (!std::is_sorted(v.begin(), v.end())) radix_sort_keys(v, 3 * l);
  }
  for (int i = 0; i < nl; ++i) {
    const auto& v = sorted[i];
    for (size_t c = 1; c < v.size(); ++c)
      if (v[c].first == v[c - 1].first) {
        char b[128];
        snprintf(b, sizeof b, "duplicate cell at level %d", lmin + i);
        return fail(AFMM_E_INVALID_ARG, b);
      }
  }

  T.lmax = std::max(T.lmax, lmax);
  T.lmin_all = std::min(T.lmin_all, lmin);
  std::vector<uint64_t> keys{0}, next;  // this hierarchy's cells at the current level
  for (int l = 0; l <= lmax; ++l) {
    HostLevel& L = T.lv[l];
    const int32_t base = L.n();
    const int32_t rbase = L.nref();
    const size_t n = keys.size();
    std::vector<uint8_t> ref(n, 1);
    std::vector<int32_t> slot(n, -1);
    const int parts = parts_for((int64_t)n, 4096);
    std::vector<int64_t> bad((size_t)parts, -1);  // first failing cell of each range, and how it failed
    std::vector<int> badkind((size_t)parts, 0);
    if (l >= lmin) {
      const int i = l - lmin;
      const auto& v = sorted[i];
      if (v.size() != n) {
        char b[160];
        snprintf(b, sizeof b, "level %d has %zu cells, the refined cells of level %d own %zu", l, v.size(), l - 1,
                 n);
        return fail(AFMM_E_INCOMPLETE_OCT, b);
      }
      parallel_ranges((int64_t)n, parts, [&](int64_t cb, int64_t ce, int part) {
        for (int64_t c = cb; c < ce; ++c) {
          if (v[(size_t)c].first != keys[(size_t)c]) {
            bad[(size_t)part] = c;
            return;
          }
          const int32_t ci = v[(size_t)c].second;
          ref[(size_t)c] = h.refined[off[i] + ci] ? 1 : 0;
          slot[(size_t)c] = (int32_t)(slot_base + off[i] + ci);
        }
      });
      for (int64_t c : bad)
        if (c >= 0) {
          char b[128];
          snprintf(b, sizeof b, "level %d: cell set differs from the children of refined level-%d cells", l, l - 1);
          return fail(AFMM_E_INCOMPLETE_OCT, b);
        }
      if (l == lmax)
        for (size_t c = 0; c < n; ++c)
          if (ref[c]) return fail(AFMM_E_INCOMPLETE_OCT, "refined cell at levelmax has no children");
    }
    // refined ranks in cell order: refined cells per range, then each range's first rank
    std::vector<int32_t> first((size_t)parts + 1, 0);
    parallel_ranges((int64_t)n, parts, [&](int64_t cb, int64_t ce, int part) {
      int32_t k = 0;
      for (int64_t c = cb; c < ce; ++c) k += ref[(size_t)c];
      first[(size_t)part + 1] = k;
    });
    for (int t = 0; t < parts; ++t) first[(size_t)t + 1] += first[(size_t)t];
    const int32_t nr = first[(size_t)parts];
    L.rank.resize((size_t)base + n);
    L.slot.resize((size_t)base + n);
    L.refcell.resize((size_t)rbase + nr);
    parallel_ranges((int64_t)n, parts, [&](int64_t cb, int64_t ce, int part) {
      int32_t r = rbase + first[(size_t)part];
      for (int64_t c = cb; c < ce; ++c) {
        const size_t g = (size_t)base + (size_t)c;
        L.slot[g] = slot[(size_t)c];
        if (ref[(size_t)c]) {
          L.rank[g] = r;
          L.refcell[(size_t)r] = (int32_t)g;
          ++r;
        } else {
          L.rank[g] = -1;
        }
      }
    });
    // neighbour rows of the refined cells, from the father's row, written at
    // their refined rank; the first grading violation in cell order is reported
    const size_t nb0 = L.nbr.size();
    L.nbr.resize(nb0 + (size_t)nr * 27);
    parallel_ranges((int64_t)n, parts, [&](int64_t cb, int64_t ce, int part) {
      for (int64_t c = cb; c < ce; ++c) {
        if (!ref[c]) continue;
        const int32_t gcell = base + (int32_t)c;
        int32_t* row = &L.nbr[nb0 + (size_t)(L.rank[gcell] - rbase) * 27];
        if (l == 0) {
          // periodic box: the root's 27 neighbours are its own images
          for (int e = 0; e < 27; ++e) row[e] = (e == 13 || T.periodic) ? gcell : -1;
        } else {
          const HostLevel& P = T.lv[l - 1];
          const int32_t fr = gcell >> 3, o = gcell & 7;
          const int32_t* prow = &P.nbr[(size_t)fr * 27];
          for (int e = 0; e < 27; ++e) {
            int pe = 0, co = 0;
            for (int d = 0, mul = 1; d < 3; ++d, mul *= 3) {
              const int ed = (d == 0 ? e % 3 : (d == 1 ? (e / 3) % 3 : e / 9)) - 1;
              const int td = ((o >> d) & 1) + ed;          // -1 .. 2
              const int pd = td < 0 ? -1 : (td >> 1);       // -1, 0, 0, 1
              pe += (pd + 1) * mul;
              co |= (td - 2 * pd) << d;
            }
            const int32_t Q = prow[pe];
            if (Q < 0) {
              row[e] = -1;
              continue;
            }
            const int32_t rQ = P.rank[Q];
            row[e] = rQ >= 0 ? 8 * rQ + co : -2;  // -2: covered by a coarser leaf
          }
          // strong grading rule: the father's 27 neighbours must be refined
          if (l >= lmin + 1) {
            for (int e = 0; e < 27; ++e) {
              const int32_t Q = prow[e];
              const int kind = Q >= 0 && P.rank[Q] < 0 ? 1 : Q == -2 ? 2 : 0;
              if (kind) {
                bad[part] = c;
                badkind[part] = kind;
                return;
              }
            }
          }
        }
      }
    });
    for (int t = 0; t < parts; ++t) {
      if (bad[t] < 0) continue;
      if (badkind[t] == 2) return fail(AFMM_E_NOT_GRADED, "grading rule violated");
      char b[160];
      snprintf(b, sizeof b, "level-%d cell refined next to a level-%d leaf (grading rule)", l, l - 1);
      return fail(AFMM_E_NOT_GRADED, b);
    }
    // the next level's cells: the children of the refined cells, in order
    next.assign((size_t)nr * 8, 0);
    parallel_ranges((int64_t)n, parts, [&](int64_t cb, int64_t ce, int part) {
      size_t r = (size_t)first[(size_t)part];
      for (int64_t c = cb; c < ce; ++c)
        if (ref[(size_t)c]) {
          for (uint64_t o = 0; o < 8; ++o) next[8 * r + o] = (keys[(size_t)c] << 3) | o;
          ++r;
        }
    });
    keys.swap(next);
  }
  T.levelmin.push_back(lmin);
  T.levelmax.push_back(lmax);
  T.slot_base.push_back(slot_base);
  T.slot_count.push_back(off[nl]);
  T.level_off.push_back(off);
  T.nslots = slot_base + off[nl];
  return AFMM_OK;
}

// Lists built on the host threads: each contiguous range of candidates fills
// its own lists, which are joined in range order (the lists are in rank order,
// whatever the thread count).
template <int NL, typename F>
static void parallel_lists(int64_t n, std::vector<int32_t>* const (&out)[NL], F&& fill) {
  const int parts = parts_for(n, 4096);
  std::vector<std::array<std::vector<int32_t>, NL>> loc((size_t)parts);
  parallel_ranges(n, parts, [&](int64_t b, int64_t e, int part) { fill(b, e, loc[(size_t)part]); });
  for (int k = 0; k < NL; ++k) {
    size_t tot = 0;
    for (auto& x : loc) tot += x[k].size();
    out[k]->clear();
    out[k]->reserve(tot);
    for (auto& x : loc) out[k]->insert(out[k]->end(), x[k].begin(), x[k].end());
  }
}

static void build_groups(Topology& T) {
  for (int l = 1; l <= T.lmax; ++l) {
    const HostLevel& P = T.lv[l - 1];
    const HostLevel& C = T.lv[l];
    auto& lg = T.leafgrp[l];
    std::vector<int32_t>* const g4[4] = {&lg, &T.m2lgrp[l], &T.upleaf[l - 1], &T.upmix[l - 1]};
    parallel_lists<4>(P.nref(), g4, [&](int64_t b, int64_t e, std::array<std::vector<int32_t>, 4>& o4) {
      for (int32_t r = (int32_t)b; r < (int32_t)e; ++r) {
        bool leaf = false, refd = false;
        for (int o = 0; o < 8; ++o) {
          if (C.rank[8 * r + o] < 0) leaf = true;
          else refd = true;
        }
        if (leaf) o4[0].push_back(r);
        if (refd && l >= 3) o4[1].push_back(r);
        o4[refd ? 3 : 2].push_back(r);
      }
    });
    // groups whose near candidates (children of the 27 neighbours of F)
    // include a refined level-l cell: their near-field M2P runs apart
    std::vector<int32_t>* const g2[2] = {&T.nmgrp[l], &T.adjvgrp[l]};
    parallel_lists<2>((int64_t)lg.size(), g2, [&](int64_t b, int64_t e, std::array<std::vector<int32_t>, 2>& o2) {
      for (int64_t i = b; i < e; ++i) {
        const int32_t r = lg[(size_t)i];
        bool any = false, coarse = false;
        const int32_t* nb = &P.nbr[(size_t)r * 27];
        for (int e2 = 0; e2 < 27; ++e2) {
          const int32_t q = nb[e2];
          if (q < 0) continue;
          if (P.rank[q] < 0) {
            coarse = true;
            continue;
          }
          for (int op = 0; op < 8 && !any; ++op) any = C.rank[8 * P.rank[q] + op] >= 0;
        }
        if (any) o2[0].push_back(r);
        if (any || coarse) o2[1].push_back(r);
      }
    });
  }
}

// ---------------------------------------------------------------------------
// work counts (algorithmic, for plan_info and the roofline)

static inline int ax_of(int e, int d) { return (d == 0 ? e % 3 : (d == 1 ? (e / 3) % 3 : e / 9)) - 1; }

static int64_t binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  int64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// Per-level algorithmic work of one synchronous solve (useful terms only).
struct WorkCounts {
  double m2l_flops[kMaxLevel] = {}, leaf_flops[kMaxLevel] = {}, up_flops[kMaxLevel] = {};
  double m2l_bytes[kMaxLevel] = {}, leaf_bytes[kMaxLevel] = {}, up_bytes[kMaxLevel] = {};
  double m2p_flops[kMaxLevel] = {}, m2p_bytes[kMaxLevel] = {};  // intermediate field (MFMA kernel)
  double l2l_flops[kMaxLevel] = {}, l2l_bytes[kMaxLevel] = {};  // ShiftLocal chain step
  int64_t m2l_targets = 0, m2l_pairs = 0, m2p = 0, p2p = 0, nm2p = 0, nst = 0, leaves = 0;
  double flops_m2l = 0, flops_m2p = 0, flops_p2p = 0, flops_updown = 0;
};

// Geometry of the pair counts, as bit masks over child octants: far[oF][e]
// has bit op when child op of the grandfather's neighbour e is in the
// interaction list of a father with octant oF (not touching it); adj[e][op]
// has bit o when child op of the father's neighbour e touches target child o,
// self[e][op] when it is that child.
struct PairMasks {
  uint8_t far[8][27] = {}, adj[27][8] = {}, self[27][8] = {};
  PairMasks() {
    for (int e = 0; e < 27; ++e)
      for (int op = 0; op < 8; ++op)
        for (int o = 0; o < 8; ++o) {
          int dm = 0;
          for (int d = 0; d < 3; ++d) dm = std::max(dm, std::abs(2 * ax_of(e, d) + ((op >> d) & 1) - ((o >> d) & 1)));
          if (dm > 1) far[o][e] |= (uint8_t)(1u << op);
          if (dm <= 1) adj[e][op] |= (uint8_t)(1u << o);
          if (dm == 0) self[e][op] |= (uint8_t)(1u << o);
        }
  }
};

static void count_work(const Topology& T, int p, bool mixed, int f64, WorkCounts& W) {
  static const PairMasks PM;
  const int K = nmi(p), K1 = nmi(p - 1);
  const double tri = (double)binom(p + 6, 6);
  const double fm2p = 2.0 * (K + 3.0 * K1), fp2p = 23.0, fl2p = 2.0 * (K + 3.0 * K1);
  double m2m_terms = 0;
  for (int a = 0; a <= p; ++a)
    for (int b = 0; a + b <= p; ++b)
      for (int c = 0; a + b + c <= p; ++c) m2m_terms += (a + 1) * (b + 1) * (c + 1);
  // interaction-list sources of group F (refined rank at level l-1): how many
  // are refined (multipole sources) and how many are leaves
  auto il_count = [&](int l, int32_t F, int64_t& refined, int64_t& leaf) {
    refined = leaf = 0;
    if (l < 2) return;
    const HostLevel& L1 = T.lv[l - 1];
    const HostLevel& L2 = T.lv[l - 2];
    const int32_t cF = L1.refcell[F];
    const int32_t G = cF >> 3, oF = cF & 7;
    for (int e = 0; e < 27; ++e) {
      const int32_t Q = L2.nbr[(size_t)G * 27 + e];
      if (Q < 0) continue;
      const uint8_t m = PM.far[oF][e];
      const int32_t base = 8 * L2.rank[Q];
      for (int op = 0; op < 8; ++op)
        if (m >> op & 1) ++(L1.rank[base + op] >= 0 ? refined : leaf);
    }
  };
  // upward: one M2M (or P2M) per child of every refined cell at levels >= 2
  for (int f = 2; f < T.lmax; ++f) {
    const double nr = T.lv[f].nref();
    W.up_flops[f] = 2.0 * 8.0 * m2m_terms * nr;
    W.up_bytes[f] = nr * K * 8.0 * (mixed && f >= f64 ? 1.5 : 1.0) + T.lv[f + 1].nref() * K * 8.0 +
                    T.lv[f + 1].n() * (8.0 + 4.0);
    W.flops_updown += W.up_flops[f];
  }
  for (int f = 3; f <= T.lmax; ++f) {
    const HostLevel& L1 = T.lv[f - 1];
    const HostLevel& L0 = T.lv[f];
    const double cs = (mixed && f > f64) ? 4.0 : 8.0;
    const auto& grp = T.m2lgrp[f];
    const int parts = parts_for((int64_t)grp.size(), 1024);  // a group is ~500 checks
    std::vector<std::array<int64_t, 3>> acc(parts, std::array<int64_t, 3>{});
    parallel_ranges((int64_t)grp.size(), parts, [&](int64_t gb, int64_t ge, int part) {
      std::array<int64_t, 3>& a = acc[part];  // pairs, monopole pairs, targets
      for (int64_t i = gb; i < ge; ++i) {
        const int32_t F = grp[i];
        int nt = 0;
        for (int o = 0; o < 8; ++o) nt += L0.rank[8 * F + o] >= 0;
        int64_t nr, nl;
        il_count(f, F, nr, nl);
        a[2] += nt;
        a[0] += nr * nt;
        a[1] += nl * nt;
      }
    });
    int64_t pairs = 0, mono = 0, nt_all = 0;
    for (const auto& a : acc) pairs += a[0], mono += a[1], nt_all += a[2];
    const double ng = (double)T.m2lgrp[f].size();
    W.m2l_targets += nt_all;
    W.m2l_pairs += pairs + mono;
    W.m2l_flops[f] = 2.0 * tri * (double)pairs + 2.0 * K * (double)mono;
    W.l2l_flops[f] = f - 1 >= 3 ? 2.0 * tri * (double)nt_all : 0.0;
    W.l2l_bytes[f] = f - 1 >= 3 ? ng * K * cs + 2.0 * (double)nt_all * K * cs : 0.0;
    W.flops_m2l += 2.0 * tri * (double)pairs + 2.0 * K * (double)mono;
    W.flops_updown += (f - 1 >= 3 ? 2.0 * tri * (double)nt_all : 0.0);
    // unique data: source multipoles of level f-1, parent and output expansions, topology
    W.m2l_bytes[f] = (double)L1.nref() * K * cs + ng * K * cs + (double)nt_all * K * cs + ng * 4.0 +
                     (double)T.lv[f - 2].nref() * 27.0 * 4.0 + (double)L1.n() * (4.0 + 8.0);
  }
  for (int l = 1; l <= T.lmax; ++l) {
    const HostLevel& L1 = T.lv[l - 1];
    const HostLevel& L0 = T.lv[l];
    const double cs = (mixed && (l - 1) > f64) ? 4.0 : 8.0;
    const auto& grp = T.leafgrp[l];
    const int parts = parts_for((int64_t)grp.size(), 1024);  // a group is ~500 checks
    std::vector<std::array<int64_t, 6>> acc(parts, std::array<int64_t, 6>{});
    parallel_ranges((int64_t)grp.size(), parts, [&](int64_t gb, int64_t ge, int part) {
      int64_t m2p = 0, p2p = 0, p2p_il = 0, nm2p = 0, nst = 0, leaves = 0;
      for (int64_t i = gb; i < ge; ++i) {
        const int32_t F = grp[i];
        unsigned tgt = 0;  // leaf children of F: the targets
        for (int o = 0; o < 8; ++o) tgt |= (L0.rank[8 * F + o] < 0 ? 1u : 0u) << o;
        const int nt = __builtin_popcount(tgt);
        leaves += nt;
        int64_t nr, nl;
        il_count(l, F, nr, nl);
        m2p += nr * nt;
        p2p_il += nl * nt;
        const int32_t* nb = &L1.nbr[(size_t)F * 27];
        for (int e = 0; e < 27; ++e) {
          const int32_t q = nb[e];
          if (q < 0) continue;
          const int32_t rq = L1.rank[q];
          if (rq < 0) {
            p2p += nt;  // a leaf one level coarser: P2P with every target
            continue;
          }
          for (int op = 0; op < 8; ++op) {
            const unsigned t = tgt & ~(unsigned)PM.self[e][op];
            if (L0.rank[8 * rq + op] < 0) {
              p2p += __builtin_popcount(t);  // leaf candidate: P2P with every other target
              continue;
            }
            const int na = __builtin_popcount(t & PM.adj[e][op]);
            p2p += 8 * na;  // touching refined candidate: nearest field from its 8 children
            nst += 8 * na;
            nm2p += __builtin_popcount(t & ~(unsigned)PM.adj[e][op]);
          }
        }
      }
      acc[part] = {m2p, p2p, p2p_il, nm2p, nst, leaves};
    });
    int64_t m2p = 0, p2p = 0, p2p_il = 0, nm2p = 0, nst = 0, leaves = 0;
    for (const auto& a : acc)
      m2p += a[0], p2p += a[1], p2p_il += a[2], nm2p += a[3], nst += a[4], leaves += a[5];
    W.m2p += m2p;
    W.p2p += p2p + p2p_il;
    W.nm2p += nm2p;
    W.nst += nst;
    W.leaves += leaves;
    const double far = (l - 1 >= 3) ? fl2p * (double)leaves : 0.0;
    W.m2p_flops[l] = fm2p * (double)m2p + fp2p * (double)p2p_il;
    W.leaf_flops[l] = fm2p * (double)nm2p + fp2p * (double)p2p + far;
    W.flops_m2p += fm2p * (double)(m2p + nm2p);
    W.flops_p2p += fp2p * (double)(p2p + p2p_il);
    W.flops_updown += far;
    const double ng = (double)T.leafgrp[l].size();
    const double nnext = l + 1 <= T.lmax ? (double)T.lv[l + 1].n() : 0.0;
    // unique data touched: intermediate sources of level l-1 and the partials it writes
    W.m2p_bytes[l] = (double)L1.nref() * K * cs + 8.0 * (double)L1.n() + 4.0 * (double)L1.n() + ng * 32.0 * cs +
                     108.0 * (double)(l >= 2 ? T.lv[l - 2].nref() : 0);
    W.leaf_bytes[l] = ng * K * cs + (double)L0.nref() * K * cs + ng * 32.0 * cs +
                      8.0 * ((double)L1.n() + (double)L0.n() + nnext) + 32.0 * (double)leaves +
                      4.0 * ((double)L1.n() + (double)L0.n()) + 108.0 * ng;
  }
}

// ---------------------------------------------------------------------------
// translation tables

// Taylor coefficients of 1/|R|:  |g| r^2 a_g = -(2|g|-1) sum_i R_i a_{g-e_i} - (|g|-1) sum_i a_{g-2e_i}
// (obtained by matching powers of t in |R+t|^2 E f = -(R.t + |t|^2) f, E the Euler operator).
static void dtilde(int p, const long double R[3], long double* D, const std::vector<int>& mi) {
  const int K = nmi(p);
  std::vector<long double> a(K);
  const long double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
  for (int g = 0; g < K; ++g) {
    const int ga[3] = {mi[4 * g], mi[4 * g + 1], mi[4 * g + 2]};
    const int n = mi[4 * g + 3];
    if (n == 0) {
      a[g] = 1.0L / std::sqrt(r2);
      continue;
    }
    long double s1 = 0, s2 = 0;
    for (int i = 0; i < 3; ++i) {
      int b[3] = {ga[0], ga[1], ga[2]};
      if (b[i] >= 1) {
        b[i] -= 1;
        s1 += R[i] * a[mi_index(b[0], b[1], b[2])];
        if (b[i] >= 1) {
          b[i] -= 1;
          s2 += a[mi_index(b[0], b[1], b[2])];
        }
      }
    }
    a[g] = (-(2.0L * n - 1.0L) * s1 - (n - 1.0L) * s2) / (n * r2);
  }
  // D~_g = d^g(-1/r) = -g! a_g
  for (int g = 0; g < K; ++g) {
    long double f = 1;
    for (int i = 0; i < 3; ++i)
      for (int k = 2; k <= mi[4 * g + i]; ++k) f *= k;
    D[g] = -f * a[g];
  }
}

struct HostTables {
  int p = 0, K = 0;
  std::vector<int> mi;          // [K][4]
  std::vector<int16_t> sumidx;  // [K][K]
  std::vector<int16_t> up;      // [K][3]
  std::vector<double> Dil, Dsame, cfac2, cfacn, l2lw, l2p, binom;
  std::vector<int32_t> taps;        // [8][189]
  std::vector<int16_t> m2p_off;     // [steps][64]
  std::vector<int16_t> m2l_off;     // [steps][64]
  std::vector<int32_t> m2m_start, m2m_list;
  std::vector<double> m2m_w;
  std::vector<int32_t> m2mT_start, m2mT_list, tapsT;
  std::vector<double> m2mT_w;
  std::vector<int32_t> m2l_tinfo;   // [NT][2]
  std::vector<int16_t> adj_m2p_off, adj_m2l_off;
  std::vector<int32_t> l2lT_start, l2lT_list;
  std::vector<double> l2lT_w;
  std::vector<double> nearA;        // [2][near_ksteps][64] near-field operator (A lane order)
};

static long double ipow(long double x, int n) {
  long double r = 1;
  for (int i = 0; i < n; ++i) r *= x;
  return r;
}
static long double fact(int n) {
  long double r = 1;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}

static void build_tables(int p, HostTables& H) {
  const int K = nmi(p);
  H.p = p;
  H.K = K;
  H.mi.assign(4 * K, 0);
  for (int n = 0; n <= p; ++n)
    for (int a = n; a >= 0; --a)
      for (int b = n - a; b >= 0; --b) {
        const int c = n - a - b, g = mi_index(a, b, c);
        H.mi[4 * g] = a;
        H.mi[4 * g + 1] = b;
        H.mi[4 * g + 2] = c;
        H.mi[4 * g + 3] = n;
      }
  H.sumidx.assign((size_t)K * K, -1);
  H.up.assign(3 * K, -1);
  for (int b = 0; b < K; ++b)
    for (int a = 0; a < K; ++a)
      if (H.mi[4 * a + 3] + H.mi[4 * b + 3] <= p)
        H.sumidx[(size_t)b * K + a] =
            (int16_t)mi_index(H.mi[4 * a] + H.mi[4 * b], H.mi[4 * a + 1] + H.mi[4 * b + 1], H.mi[4 * a + 2] + H.mi[4 * b + 2]);
  for (int a = 0; a < K; ++a)
    if (H.mi[4 * a + 3] < p)
      for (int i = 0; i < 3; ++i)
        H.up[3 * a + i] = (int16_t)mi_index(H.mi[4 * a] + (i == 0), H.mi[4 * a + 1] + (i == 1), H.mi[4 * a + 2] + (i == 2));
  std::vector<long double> D(K);
  H.Dil.assign((size_t)kNumD * 8 * K, 0.0);
  H.Dsame.assign((size_t)kNumD * K, 0.0);
  for (int dz = -3; dz <= 3; ++dz)
    for (int dy = -3; dy <= 3; ++dy)
      for (int dx = -3; dx <= 3; ++dx) {
        const int di = (dx + 3) + 7 * (dy + 3) + 49 * (dz + 3);
        for (int o = 0; o < 8; ++o) {
          const long double R[3] = {-2.0L * dx + ((o & 1) - 0.5L), -2.0L * dy + (((o >> 1) & 1) - 0.5L),
                                    -2.0L * dz + (((o >> 2) & 1) - 0.5L)};
          dtilde(p, R, D.data(), H.mi);
          for (int g = 0; g < K; ++g) H.Dil[((size_t)di * 8 + o) * K + g] = (double)D[g];
        }
        if (dx == 0 && dy == 0 && dz == 0) continue;
        const long double R[3] = {(long double)dx, (long double)dy, (long double)dz};
        dtilde(p, R, D.data(), H.mi);
        for (int g = 0; g < K; ++g) H.Dsame[(size_t)di * K + g] = (double)D[g];
      }
  H.cfac2.resize(K);
  H.cfacn.resize(K);
  for (int a = 0; a < K; ++a) {
    const int n = H.mi[4 * a + 3];
    const long double af = fact(H.mi[4 * a]) * fact(H.mi[4 * a + 1]) * fact(H.mi[4 * a + 2]);
    const long double sg = (n & 1) ? -1.0L : 1.0L;
    H.cfacn[a] = (double)(1.0L / ipow(2.0L, n));
    H.cfac2[a] = (double)(sg * ipow(2.0L, n) / af);
  }
  // L2L weights: L~_b[y] = 2^(-1-|b|) sum_g u^g/g! L~_{b+g}[F], u = (o - 1/2)/2, stored per |b|
  H.l2lw.assign((size_t)8 * (p + 1) * K, 0.0);
  H.l2p.assign((size_t)8 * 4 * K, 0.0);
  for (int o = 0; o < 8; ++o) {
    const long double u[3] = {((o & 1) - 0.5L) / 2, (((o >> 1) & 1) - 0.5L) / 2, (((o >> 2) & 1) - 0.5L) / 2};
    for (int nb = 0; nb <= p; ++nb)
      for (int g = 0; g < nmi(p - nb); ++g) {
        const int* gg = &H.mi[4 * g];
        H.l2lw[((size_t)o * (p + 1) + nb) * K + g] =
            (double)(ipow(u[0], gg[0]) * ipow(u[1], gg[1]) * ipow(u[2], gg[2]) / (fact(gg[0]) * fact(gg[1]) * fact(gg[2])) /
                     ipow(2.0L, 1 + nb));
      }
    // L2P: phi~ = 1/2 sum_b L~_b u^b/b!,  a~_i = -1/4 sum_{b_i>0} L~_b u^(b-e_i)/(b-e_i)!
    for (int b = 0; b < K; ++b) {
      const int* bb = &H.mi[4 * b];
      const long double bf = fact(bb[0]) * fact(bb[1]) * fact(bb[2]);
      H.l2p[((size_t)o * 4 + 0) * K + b] = (double)(0.5L * ipow(u[0], bb[0]) * ipow(u[1], bb[1]) * ipow(u[2], bb[2]) / bf);
      for (int i = 0; i < 3; ++i) {
        if (bb[i] == 0) continue;
        int c[3] = {bb[0], bb[1], bb[2]};
        c[i] -= 1;
        H.l2p[((size_t)o * 4 + 1 + i) * K + b] =
            (double)(-0.25L * ipow(u[0], c[0]) * ipow(u[1], c[1]) * ipow(u[2], c[2]) / (fact(c[0]) * fact(c[1]) * fact(c[2])));
      }
    }
  }
  // Near-field operator of a group (target-level units): P2P kernel values
  // phi~ = -1/|R|, a~ = -R/|R|^3 at R = target - source for the 216 same-level
  // candidates (the target itself excluded) and the 27 coarse neighbours, then
  // the L2P weights.  Row 16 t + (lane & 15), column 4 kb + (lane >> 4).
  {
    const int NKB = near_ksteps(p);
    H.nearA.assign((size_t)2 * NKB * 64, 0.0);
    for (int t = 0; t < 2; ++t)
      for (int kb = 0; kb < NKB; ++kb)
        for (int lane = 0; lane < 64; ++lane) {
          const int R = 16 * t + (lane & 15), k = 4 * kb + (lane >> 4);
          const int c = R >> 3, o = R & 7;
          double v = 0.0;
          long double r[3];
          bool pair = false;
          if (k < kNearLeafCols) {
            const int e = k >> 3, op = k & 7;
            if (!(e == 13 && op == o)) {
              for (int d = 0; d < 3; ++d) {
                const int ed = (d == 0 ? e % 3 : d == 1 ? (e / 3) % 3 : e / 9) - 1;
                r[d] = (long double)(((o >> d) & 1) - 2 * ed - ((op >> d) & 1));
              }
              pair = true;
            }
          } else if (k < kNearLeafCols + kNearCoarseCols) {
            const int e = k - kNearLeafCols;
            for (int d = 0; d < 3; ++d) {
              const int ed = (d == 0 ? e % 3 : d == 1 ? (e / 3) % 3 : e / 9) - 1;
              r[d] = (long double)((o >> d) & 1) - 0.5L - 2.0L * ed;
            }
            pair = true;
          } else if (k < kNearLeafCols + kNearCoarseCols + K) {
            v = H.l2p[((size_t)o * 4 + c) * K + (k - kNearLeafCols - kNearCoarseCols)];
          }
          if (pair) {
            const long double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            const long double inv = 1.0L / std::sqrt(r2);
            v = (double)(c == 0 ? -inv : -r[c - 1] * inv * inv * inv);
          }
          H.nearA[((size_t)t * NKB + kb) * 64 + lane] = v;
        }
  }
  // M2M (upward) entries per coefficient a: k <= a, weight C(a,k) 4^-|a-k| 2^-|k|,
  // sign pattern = parity of a - k (applied through the signed child sums)
  H.m2m_start.assign(K + 1, 0);
  H.m2m_list.clear();
  H.m2m_w.clear();
  for (int a = 0; a < K; ++a) {
    H.m2m_start[a] = (int32_t)H.m2m_list.size();
    const int* aa = &H.mi[4 * a];
    for (int k0 = 0; k0 <= aa[0]; ++k0)
      for (int k1 = 0; k1 <= aa[1]; ++k1)
        for (int k2 = 0; k2 <= aa[2]; ++k2) {
          const int v0 = aa[0] - k0, v1 = aa[1] - k1, v2 = aa[2] - k2;
          const int q = (v0 & 1) | ((v1 & 1) << 1) | ((v2 & 1) << 2);
          H.m2m_list.push_back(mi_index(k0, k1, k2) | (q << 12));
          H.m2m_w.push_back((double)((long double)binom(aa[0], k0) * binom(aa[1], k1) * binom(aa[2], k2) /
                                     ipow(2.0L, 2 * (v0 + v1 + v2) + k0 + k1 + k2)));
        }
  }
  H.m2m_start[K] = (int32_t)H.m2m_list.size();
  // the same entries grouped by k, for the transposed M2M of the adjoint pass
  H.m2mT_start.assign(K + 1, 0);
  H.m2mT_list.clear();
  H.m2mT_w.clear();
  for (int k = 0; k < K; ++k) {
    H.m2mT_start[k] = (int32_t)H.m2mT_list.size();
    for (int a = 0; a < K; ++a)
      for (int j = H.m2m_start[a]; j < H.m2m_start[a + 1]; ++j)
        if ((H.m2m_list[j] & 4095) == k) {
          H.m2mT_list.push_back(a | (H.m2m_list[j] >> 12) << 12);
          H.m2mT_w.push_back(H.m2m_w[j]);
        }
  }
  H.m2mT_start[K] = (int32_t)H.m2mT_list.size();
  H.binom.assign((kPMax + 1) * (kPMax + 1), 0.0);
  for (int n = 0; n <= kPMax; ++n)
    for (int k = 0; k <= n; ++k) H.binom[n * (kPMax + 1) + k] = (double)binom(n, k);
  // taps of each parity class: neighbour e of G, child o' -> d = 2e + o' - o_F with |d|_inf >= 2
  H.taps.clear();
  for (int oF = 0; oF < 8; ++oF) {
    int cnt = 0;
    for (int e = 0; e < 27; ++e)
      for (int op = 0; op < 8; ++op) {
        int d[3], dm = 0;
        for (int a = 0; a < 3; ++a) {
          d[a] = 2 * ax_of(e, a) + ((op >> a) & 1) - ((oF >> a) & 1);
          dm = std::max(dm, std::abs(d[a]));
        }
        if (dm <= 1) continue;
        const int di = (d[0] + 3) + 7 * (d[1] + 3) + 49 * (d[2] + 3);
        H.taps.push_back(e | (op << 5) | (di << 8));
        ++cnt;
      }
    (void)cnt;
  }
  // transposed taps of each source octant os: groups F = child oF of the
  // neighbour e of the source's father, d = s - F = os - oF - 2e, |d|_inf >= 2
  H.tapsT.clear();
  for (int os = 0; os < 8; ++os)
    for (int e = 0; e < 27; ++e)
      for (int oF = 0; oF < 8; ++oF) {
        int d[3], dm = 0;
        for (int a = 0; a < 3; ++a) {
          d[a] = ((os >> a) & 1) - ((oF >> a) & 1) - 2 * ax_of(e, a);
          dm = std::max(dm, std::abs(d[a]));
        }
        if (dm <= 1) continue;
        const int di = (d[0] + 3) + 7 * (d[1] + 3) + 49 * (d[2] + 3);
        H.tapsT.push_back(e | (oF << 5) | (di << 8));
      }
  // MFMA A-operand offsets into the staged D~ rows (sD[o][g], row stride KS, zero slot 8 KS)
  const int KP = (K + 3) & ~3, KS = dstage_ks(p), ZERO = 8 * KS, K1 = nmi(p - 1);
  auto deg = [&](int idx) { return H.mi[4 * idx + 3]; };
  H.m2p_off.clear();
  for (int rt = 0; rt < 2; ++rt) {
    const int steps = rt == 0 ? KP / 4 : (K1 + 3) / 4;
    for (int kb = 0; kb < steps; ++kb)
      for (int lane = 0; lane < 64; ++lane) {
        const int i = lane & 15, k = 4 * kb + (lane >> 4);
        const int c = 2 * rt + (i >> 3), o = i & 7;  // c: 0 phi, 1..3 a_x..a_z
        int v = ZERO;
        if (c == 0 && k < K) v = o * KS + k;
        if (c > 0 && k < K1) v = o * KS + H.up[3 * k + (c - 1)];
        H.m2p_off.push_back((int16_t)v);
      }
  }
  // adjoint: transposed L2L pairs (b <= c componentwise, g = c - b) per c
  H.l2lT_start.assign(K + 1, 0);
  H.l2lT_list.clear();
  for (int c = 0; c < K; ++c) {
    H.l2lT_start[c] = (int32_t)H.l2lT_list.size();
    for (int b = 0; b < K; ++b) {
      const int g0 = H.mi[4 * c] - H.mi[4 * b], g1 = H.mi[4 * c + 1] - H.mi[4 * b + 1], g2 = H.mi[4 * c + 2] - H.mi[4 * b + 2];
      if (g0 < 0 || g1 < 0 || g2 < 0) continue;
      H.l2lT_list.push_back(b | (mi_index(g0, g1, g2) << 8) | (H.mi[4 * b + 3] << 16) |
                            (((g0 & 1) | (g1 & 1) << 1 | (g2 & 1) << 2) << 24));
    }
  }
  H.l2lT_start[K] = (int32_t)H.l2lT_list.size();
  // weight of child 7 (offset components all +1/4); child o differs by the sign
  // (-1)^popcount(~o & parity(c - b)), applied to the children's bars on the device
  H.l2lT_w.assign(H.l2lT_list.size(), 0.0);
  for (size_t j = 0; j < H.l2lT_list.size(); ++j) {
    const int g = (H.l2lT_list[j] >> 8) & 255, nb = (H.l2lT_list[j] >> 16) & 255;
    H.l2lT_w[j] = H.l2lw[((size_t)7 * (p + 1) + nb) * K + g];
  }
  // adjoint: transposed M2P, rows a (tiles of 16), k = 8 g + kb -> (child o, quantity q)
  {
    const int RT = (K + 15) / 16;
    H.adj_m2p_off.clear();
    for (int rt = 0; rt < RT; ++rt)
      for (int kb = 0; kb < 8; ++kb)
        for (int lane = 0; lane < 64; ++lane) {
          const int a = 16 * rt + (lane & 15), j = 8 * (lane >> 4) + kb, o = j >> 2, q = j & 3;
          int v = ZERO;
          if (a < K && q == 0) v = o * KS + a;
          if (a < K1 && q > 0) v = o * KS + H.up[3 * a + (q - 1)];
          H.adj_m2p_off.push_back((int16_t)v);
        }
    // transposed M2L, rows a, k = b = 4 kb + g, offsets within one D~ row (K = its zero)
    H.adj_m2l_off.clear();
    for (int rt = 0; rt < RT; ++rt) {
      int d = 0;
      while (nmi(d) <= 16 * rt) ++d;
      const int ks = (nmi(p - d) + 3) / 4;
      for (int kb = 0; kb < ks; ++kb)
        for (int lane = 0; lane < 64; ++lane) {
          const int a = 16 * rt + (lane & 15), b = 4 * kb + (lane >> 4);
          int v = K;
          if (a < K && b < K && deg(a) + deg(b) <= p)
            v = mi_index(H.mi[4 * a] + H.mi[4 * b], H.mi[4 * a + 1] + H.mi[4 * b + 1], H.mi[4 * a + 2] + H.mi[4 * b + 2]);
          H.adj_m2l_off.push_back((int16_t)v);
        }
    }
  }
  const int NT = (8 * K + 15) / 16;
  H.m2l_tinfo.assign(2 * NT, 0);
  H.m2l_off.clear();
  int step = 0;
  for (int T = 0; T < NT; ++T) {
    const int ks = (nmi(p - deg(2 * T)) + 3) / 4;
    H.m2l_tinfo[2 * T] = ks;
    H.m2l_tinfo[2 * T + 1] = step;
    step += ks;
    for (int kb = 0; kb < ks; ++kb)
      for (int lane = 0; lane < 64; ++lane) {
        const int R = 16 * T + (lane & 15), k = 4 * kb + (lane >> 4);
        const int b = R >> 3, o = R & 7;
        int v = ZERO;
        if (b < K && k < K && deg(k) + deg(b) <= p)
          v = o * KS + mi_index(H.mi[4 * k] + H.mi[4 * b], H.mi[4 * k + 1] + H.mi[4 * b + 1], H.mi[4 * k + 2] + H.mi[4 * b + 2]);
        H.m2l_off.push_back((int16_t)v);
      }
  }
}

// The translation tables depend on the order only: built once per order and
// shared (read only) by every plan of the process.
static std::shared_ptr<const HostTables> tables_for(int p) {
  static std::mutex mu;
  static std::shared_ptr<const HostTables> cache[kPMax + 1];
  std::lock_guard<std::mutex> lock(mu);
  if (!cache[p]) {
    auto t = std::make_shared<HostTables>();
    build_tables(p, *t);
    cache[p] = t;
  }
  return cache[p];
}

// Potential at the centre of a uniform unit cube of unit mass, up to -G/h:
// C = integral over [-1/2, 1/2]^3 of 1/|r|.  Splitting the cube into the six
// pyramids from its centre to its faces and integrating along the rays
// r = t (1/2, y, z), 0 <= t <= 1 (volume element t^2/2 dt dy dz, so the radial
// integral of 1/|r| gives 1/2 times 1/2) leaves a smooth surface integral per
// face; with its four symmetric quarters,
// C = 6 * int_0^{1/2} int_0^{1/2} (1/4 + y^2 + z^2)^(-1/2) dy dz,
// computed with a tensor Gauss-Legendre rule whose nodes come from Newton
// iterations on the Legendre polynomial.
static double cube_self_constant() {
  constexpr int N = 48;
  long double x[N], w[N];
  for (int i = 0; i < N; ++i) {
    long double t = std::cos(3.14159265358979323846264338327950288L * (i + 0.75L) / (N + 0.5L));
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1.0L, p1 = t;
      for (int k = 2; k <= N; ++k) {
        const long double p2 = ((2.0L * k - 1.0L) * t * p1 - (k - 1.0L) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const long double dp = N * (t * p1 - p0) / (t * t - 1.0L);
      const long double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-19L) {
        x[i] = t;
        w[i] = 2.0L / ((1.0L - t * t) * dp * dp);
        break;
      }
      x[i] = t;
      w[i] = 2.0L / ((1.0L - t * t) * dp * dp);
    }
  }
  long double sum = 0.0L;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      const long double y = 0.25L * (x[i] + 1.0L), z = 0.25L * (x[j] + 1.0L);  // nodes on [0, 1/2]
      sum += w[i] * w[j] / std::sqrt(0.25L + y * y + z * z);
    }
  return (double)(6.0L * 0.0625L * sum);  // (1/4)^2: the Jacobian of [-1, 1]^2 -> [0, 1/2]^2
}

}  // namespace afmm

// ---------------------------------------------------------------------------
// plan

using namespace afmm;

struct afmm_plan {
  afmm_options opt{};
  int K = 0;
  Topology topo;
  std::shared_ptr<const HostTables> tabs;  // shared by every plan of the same order
  LevelDev lv[kMaxLevel + 1];
  int32_t* d_leafgrp[kMaxLevel] = {};
  int32_t* d_m2lgrp[kMaxLevel] = {};
  int32_t* d_nmgrp[kMaxLevel] = {};
  int32_t* d_adjvgrp[kMaxLevel] = {};
  int32_t* d_upleaf[kMaxLevel] = {};  // upward lists (Topology::upleaf / upmix)
  int32_t* d_upmix[kMaxLevel] = {};
  void* d_nmp[kMaxLevel] = {};   // near-field M2P partials of level l (leaf-kernel precision)
  // MFMA tile records of every level, one array per precision (0 FP64, 1 FP32);
  // range[l] = {precision, first tile, count}
  MfmaTiles m2p_all[2], m2l_all[2];
  MfmaTiles m2p_all2[2];            // M2P tiles of 32 groups (tile shape 2), same level ranges as below
  int m2p_range2[kMaxLevel][3] = {};
  int m2p_shape[2] = {0, 0};        // M2P tile shape per precision (afmm_options.m2p_shape)
  // Level solves (ATS, Alg. 2): the M2L / L2L work restricted to the FMM cells
  // that are ancestors of the leaves of target level l (per target level l)
  struct AtsChain {
    bool on = false;
    MfmaTiles m2l_all[2];
    int m2l_range[kMaxLevel][3] = {};
    int32_t* d_grp[kMaxLevel] = {};
    int ngrp[kMaxLevel] = {};
  } ats[kMaxLevel];
  int m2p_range[kMaxLevel][3] = {};
  int m2l_range[kMaxLevel][3] = {};
  int m2l_split[2] = {1, 1};        // tap ranges per M2L tile, per precision
  int m2p_split[2] = {1, 1};        // tap ranges per M2P tile, per precision
  LevelDev* d_lvs = nullptr;        // device copy of lv[]
  // internal side stream: the downward M2L/L2L chain runs on it concurrently
  // with the leaf-level M2P (they only share the multipoles of the upward pass)
  hipStream_t side = nullptr;
  // AFMM_GRAPH: solves replayed from captured graphs, one per (level, rebuild,
  // kept trees, caller pointers), captured on an internal stream on first use
  struct GraphEntry {
    int level;
    bool rebuild, keep;
    const double* m;
    double* phi;
    double* acc;
    hipGraph_t g;
    hipGraphExec_t x;
    uint64_t used;
  };
  std::vector<GraphEntry> graphs;
  uint64_t graph_tick = 0;
  hipStream_t cap = nullptr;
  bool capturing = false;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  MfmaTables mt;
  TablesDev<float> t32;
  TablesDev<double> t64;
  CommonDev cm;
  double* m_snap = nullptr;       // adaptive-time-step snapshot of leaf masses (slot space)
  // drifted solves (afmm_solve_drift): mass rates of the snapshot, the time of
  // each level's last rebuild, whether that rebuild recorded rates, and the
  // drifted masses a solve reads (allocated by the first drifted solve)
  double* rate_snap = nullptr;
  double* m_drift = nullptr;
  double t_snap[kMaxLevel] = {};
  bool rate_valid[kMaxLevel] = {};
  uint64_t* d_keys[kMaxLevel] = {};  // per-level Morton keys of the cells (particle-mesh calls, on first use)
  int* d_flag = nullptr;          // AFMM_CHECK_INPUT / particle-mesh calls: device flag (plan-owned)
  int* h_flag = nullptr;          // its pinned host copy
  double cself = 0.0;             // AFMM_SELF_POTENTIAL: the unit-cube constant, else 0
  // AFMM_PERIODIC: the level-2 far operator ([8][kNumD][K], level-2 units) and the
  // multipole factors (-1)^|a|/a! it is applied with (0 at order p with the quadrupole cap)
  const double* d_pfar = nullptr;
  const double* d_pfar_cf = nullptr;
  int l_first = 3;                // first FMM level with local expansions (2 with periodic boxes)
  bool snap_valid = false;
  // the per-level masses and merged multipoles on the device were computed from
  // the current snapshot m_snap (a solve that rebuilds no tree can skip them)
  bool tree_fresh = false;
  bool solved = false;            // a solve has run (the adjoint transposes the last one)
  int last_level = AFMM_ALL_LEVELS;
  int last_fresh = 0;             // levels >= this took their masses from the last call's d_mass
  int fresh_from = 1 << 20;       // after afmm_plan_replan: levels >= this take their masses from the next call
  bool adj_ready = false;         // adjoint workspace allocated
  bool adj_topo = false;          // adjoint source tiles and splits built
  size_t adj_part_elems = 0;      // FP64 elements of the adjoint's tap-split partial sets
  // source tiles of the transposed M2P (index: leaf level l) and M2L (index: FMM level f)
  int32_t* d_adjp[kMaxLevel] = {};
  int32_t* d_adjl[kMaxLevel] = {};
  // per refined rank at the source level: 1 if the group has a target child
  // (a leaf child for the M2P, a refined child for the M2L)
  uint8_t* d_adjp_live[kMaxLevel] = {};
  uint8_t* d_adjl_live[kMaxLevel] = {};
  XcdRanges xr_adjp[kMaxLevel], xr_adjl[kMaxLevel];  // their work items per XCD
  int n_adjp[kMaxLevel] = {}, n_adjl[kMaxLevel] = {};
  int s_adjp[kMaxLevel] = {}, s_adjl[kMaxLevel] = {};  // their tap splits
  double* adj_part = nullptr;     // partial sets of the split transposed translations
  struct Alloc {
    void* p;
    size_t cap;   // bytes allocated (a cached buffer may hold more than asked for)
    int dev;
    bool cached;  // returned to the buffer cache when the plan goes
  };
  std::vector<Alloc> allocs;
  size_t bytes = 0;               // bytes the plan's buffers asked for
  bool dead = false;              // sticky device error
  // sizes and work counts of the plan, counted on first use (afmm_plan_get_info,
  // profiling): a time-step loop that re-plans every few steps never asks
  mutable afmm_plan_info info{};
  mutable WorkCounts work;
  mutable std::once_flag info_once;
  // per-launch event timing (afmm_plan_set_profiling)
  bool profiling = false;
  double pending_flops = 0.0, pending_bytes = 0.0;  // work of a multi-level launch being timed
  struct Rec { int kind; int level; hipEvent_t a, b; double flops, bytes; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> event_pool;
  std::vector<afmm_stage_time> acc;
};

struct afmm_batch {
  afmm_plan* plan = nullptr;      // one plan over the forest of all hierarchies
  int32_t n = 0;
  std::vector<int64_t> base;      // [n + 1] slot offset of each hierarchy in the forest
  double* d_mass = nullptr;       // forest-wide slot arrays
  double* d_phi = nullptr;
  double* d_acc = nullptr;
  int32_t* d_leafslot = nullptr;  // forest slot of every leaf
  int32_t* d_leafhier = nullptr;  // its hierarchy
  int64_t* d_base = nullptr;
  void** d_ptrs = nullptr;        // [3][n] caller pointers (mass, phi, acc), refreshed per solve
  void** h_stage = nullptr;       // pinned [3][n] caller pointers, read by the asynchronous table upload
  hipEvent_t ev_stage = nullptr;  // recorded after that upload: h_stage may be rewritten once it completes
  int64_t nleaf = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;      // capture stream
};

namespace {

// Device buffers of destroyed plans are kept for later plans on the same
// device, up to kCacheBytes per device (the oldest go back to the driver
// first).  A hipMalloc maps new pages and a hipFree waits for the device and
// unmaps them: for a plan of a few hundred thousand cells that is several
// milliseconds, which a time-step loop that re-plans every few steps would pay
// each time.  A cached buffer is reused when it holds the request with at most
// a quarter to spare; a new one gets an eighth more than asked, so that the
// same buffer of the next plan, a little larger, still fits.  Plans with a
// device-byte cap take buffers of the exact size and free them.
constexpr size_t kCacheBytes = (size_t)2 << 30;
struct CachedBuf {
  void* p;
  size_t cap;
};
std::mutex g_cache_mu;
std::vector<std::vector<CachedBuf>> g_cache;  // per device, oldest first
std::vector<size_t> g_cache_total;

void* cache_take(int dev, size_t bytes, size_t* cap) {
  std::lock_guard<std::mutex> g(g_cache_mu);
  if (dev < 0 || (size_t)dev >= g_cache.size()) return nullptr;
  auto& v = g_cache[dev];
  const size_t hi = bytes + bytes / 4 + ((size_t)64 << 10);
  size_t best = v.size();
  for (size_t i = 0; i < v.size(); ++i)
    if (v[i].cap >= bytes && v[i].cap <= hi && (best == v.size() || v[i].cap < v[best].cap)) best = i;
  if (best == v.size()) return nullptr;
  void* p = v[best].p;
  *cap = v[best].cap;
  g_cache_total[dev] -= *cap;
  v.erase(v.begin() + (long)best);
  return p;
}

// Takes buffers that no pending device work uses any more.
void cache_put(int dev, void* p, size_t cap) {
  std::vector<void*> drop;
  {
    std::lock_guard<std::mutex> g(g_cache_mu);
    if ((size_t)dev >= g_cache.size()) {
      g_cache.resize((size_t)dev + 1);
      g_cache_total.resize((size_t)dev + 1, 0);
    }
    auto& v = g_cache[dev];
    v.push_back({p, cap});
    g_cache_total[dev] += cap;
    size_t k = 0;
    while (g_cache_total[dev] > kCacheBytes && k < v.size()) {
      drop.push_back(v[k].p);
      g_cache_total[dev] -= v[k].cap;
      ++k;
    }
    v.erase(v.begin(), v.begin() + (long)k);
  }
  for (void* q : drop) (void)hipFree(q);
}

// Returns the cached buffers of one device (dev >= 0) or of all devices.
void cache_release(int dev) {
  std::vector<void*> drop;
  {
    std::lock_guard<std::mutex> g(g_cache_mu);
    for (size_t d = 0; d < g_cache.size(); ++d) {
      if (dev >= 0 && (size_t)dev != d) continue;
      for (auto& b : g_cache[d]) drop.push_back(b.p);
      g_cache[d].clear();
      g_cache_total[d] = 0;
    }
  }
  for (void* q : drop) (void)hipFree(q);
}

// Waits for every device that holds one of the plan's cached buffers: a buffer
// goes back to the cache only once no kernel or copy can still touch it (what
// hipFree does by itself).
void sync_alloc_devices(const afmm_plan* P) {
  std::vector<int> done;
  int cur = -1;
  (void)hipGetDevice(&cur);
  for (const auto& a : P->allocs) {
    if (!a.cached || std::find(done.begin(), done.end(), a.dev) != done.end()) continue;
    done.push_back(a.dev);
    if (a.dev != cur) (void)hipSetDevice(a.dev);
    (void)hipDeviceSynchronize();
  }
  if (cur >= 0 && !done.empty()) (void)hipSetDevice(cur);
}

afmm_status dev_alloc(afmm_plan* P, void** ptr, size_t bytes) {
  *ptr = nullptr;
  if (bytes == 0) return AFMM_OK;
  if (P->opt.max_device_bytes && P->bytes + bytes > P->opt.max_device_bytes)
    return fail(AFMM_E_OUT_OF_MEMORY, "plan would exceed max_device_bytes");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(AFMM_E_DEVICE, "no current device");
  const bool cached = P->opt.max_device_bytes == 0;
  size_t cap = bytes;
  void* p = cached ? cache_take(dev, bytes, &cap) : nullptr;
  if (!p) {
    cap = cached ? (bytes + bytes / 8 + 4095) & ~(size_t)4095 : bytes;
    if (hipMalloc(&p, cap) != hipSuccess) {
      // give the cached buffers back to the driver and try once more
      (void)hipGetLastError();
      cache_release(dev);
      if (hipMalloc(&p, cap) != hipSuccess) {
        (void)hipGetLastError();
        return fail(AFMM_E_OUT_OF_MEMORY, "hipMalloc failed");
      }
    }
  }
  P->allocs.push_back({p, cap, dev, cached});
  *ptr = p;
  P->bytes += bytes;
  return AFMM_OK;
}

template <typename V>
afmm_status upload(afmm_plan* P, const std::vector<V>& v, V** out, hipStream_t st) {
  *out = nullptr;
  if (v.empty()) return AFMM_OK;
  void* p = nullptr;
  afmm_status s = dev_alloc(P, &p, v.size() * sizeof(V));
  if (s) return s;
  // the source is often a temporary: wait for the copy before it can go away
  if (hipMemcpyAsync(p, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(AFMM_E_DEVICE, "upload failed");
  *out = (V*)p;
  return AFMM_OK;
}

template <typename T>
afmm_status upload_conv(afmm_plan* P, const std::vector<double>& v, const T** out, hipStream_t st) {
  std::vector<T> w(v.begin(), v.end());
  T* d = nullptr;
  afmm_status s = upload(P, w, &d, st);
  *out = d;
  return s;
}

void drop_graphs(afmm_plan* P) {
  for (auto& e : P->graphs) {
    if (e.x) (void)hipGraphExecDestroy(e.x);
    if (e.g) (void)hipGraphDestroy(e.g);
  }
  P->graphs.clear();
}

void free_plan(afmm_plan* P) {
  if (P->side) (void)hipStreamSynchronize(P->side);
  if (P->cap) (void)hipStreamSynchronize(P->cap);
  drop_graphs(P);
  if (P->cap) (void)hipStreamDestroy(P->cap);
  P->cap = nullptr;
  sync_alloc_devices(P);
  for (const auto& a : P->allocs) {
    if (a.cached) cache_put(a.dev, a.p, a.cap);
    else (void)hipFree(a.p);
  }
  P->allocs.clear();
  if (P->h_flag) (void)hipHostFree(P->h_flag);
  P->h_flag = nullptr;
  if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
  if (P->ev_join) (void)hipEventDestroy(P->ev_join);
  if (P->side) (void)hipStreamDestroy(P->side);
  P->ev_fork = P->ev_join = nullptr;
  P->side = nullptr;
  for (auto& r : P->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  P->recs.clear();
  for (hipEvent_t e : P->event_pool) (void)hipEventDestroy(e);
  P->event_pool.clear();
}

afmm_status check_options(const afmm_options* o) {
  if (!o) return fail(AFMM_E_INVALID_ARG, "null options");
  if (o->p < 1 || o->p > kPMax) return fail(AFMM_E_UNSUPPORTED, "p must be in 1..8");
  if (o->precision != AFMM_FP64 && o->precision != AFMM_FP32_MIXED)
    return fail(AFMM_E_UNSUPPORTED, "unknown precision");
  if (o->flags & ~(AFMM_CHECK_INPUT | AFMM_SERIAL | AFMM_OVERLAP | AFMM_PAPER_QUAD_CAP | AFMM_SELF_POTENTIAL | AFMM_GRAPH |
                   AFMM_PERIODIC))
    return fail(AFMM_E_UNSUPPORTED, "unknown flag");
  if (!(o->boxlen > 0) || !std::isfinite(o->boxlen)) return fail(AFMM_E_INVALID_ARG, "boxlen must be > 0");
  if (!std::isfinite(o->G)) return fail(AFMM_E_INVALID_ARG, "G must be finite");
  if (o->tap_split < 0 || o->tap_split > 21) return fail(AFMM_E_UNSUPPORTED, "tap_split must be in 0..21");
  if (o->m2p_shape < 0 || o->m2p_shape > 3) return fail(AFMM_E_UNSUPPORTED, "m2p_shape must be in 0..3");
  return AFMM_OK;
}

void fill_info(afmm_plan_info& info, WorkCounts& W, const Topology& T, const afmm_options& o) {
  std::memset(&info, 0, sizeof info);
  info.levelmin = T.lmin_all;
  info.levelmax = T.lmax;
  info.p = o.p;
  info.K = nmi(o.p);
  info.precision = o.precision;
  info.nhier = (int32_t)T.levelmin.size();
  for (int l = 0; l <= T.lmax; ++l) {
    const HostLevel& L = T.lv[l];
    int64_t leaves = 0;
    for (int32_t c = 0; c < L.n(); ++c) leaves += (L.rank[c] < 0 && L.slot[c] >= 0);
    info.leaves_per_level[l] = leaves;
    info.nleaves += leaves;
    for (int32_t c = 0; c < L.n(); ++c)
      if (L.slot[c] >= 0) {
        ++info.ncell;
        info.nrefined += L.rank[c] >= 0;
      }
  }
  const bool mixed = o.precision == AFMM_FP32_MIXED;
  W = WorkCounts();
  count_work(T, o.p, mixed, mixed ? o.fp64_levels : 1 << 20, W);
  info.m2l_targets = W.m2l_targets;
  info.m2l_pairs = W.m2l_pairs;
  info.m2p_pairs = W.m2p;
  info.p2p_pairs = W.p2p;
  info.near_m2p_pairs = W.nm2p;
  info.nearest_pairs = W.nst;
  info.flops_m2l = W.flops_m2l;
  info.flops_m2p = W.flops_m2p;
  info.flops_p2p = W.flops_p2p;
  info.flops_updown = W.flops_updown;
  double b = 8.0 * info.nleaves;  // mass gather
  for (int l = 0; l <= T.lmax; ++l) b += W.up_bytes[l] + W.m2l_bytes[l] + W.l2l_bytes[l] + W.m2p_bytes[l] + W.leaf_bytes[l];
  info.bytes_min = b;
}

}  // namespace

extern "C" {

void afmm_options_default(afmm_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->p = 4;
  o->precision = AFMM_FP64;
  o->G = 1.0;
  o->boxlen = 1.0;
  o->flags = 0;
  o->fp64_levels = 3;
  o->tap_split = 0;
  o->max_device_bytes = 0;
  o->m2p_shape = 0;
}

const char* afmm_status_string(afmm_status s) {
  switch (s) {
    case AFMM_OK: return "ok";
    case AFMM_E_INVALID_ARG: return "invalid argument";
    case AFMM_E_NOT_GRADED: return "hierarchy not graded";
    case AFMM_E_INCOMPLETE_OCT: return "incomplete oct";
    case AFMM_E_UNSUPPORTED: return "unsupported option";
    case AFMM_E_OUT_OF_MEMORY: return "out of device memory";
    case AFMM_E_DEVICE: return "device error";
    case AFMM_E_ATS_ORDER: return "adaptive time step call order";
    case AFMM_E_NONFINITE: return "non-finite input";
    default: return "unknown status";
  }
}

const char* afmm_last_error(void) { return g_last_error.c_str(); }

static afmm_status afmm_hierarchy_check_impl(const afmm_hierarchy* h, const afmm_options* opt, afmm_plan_info* out) {
  if (!h) return fail(AFMM_E_INVALID_ARG, "null hierarchy");
  afmm_options o;
  if (opt) o = *opt;
  else afmm_options_default(&o);
  afmm_status s = check_options(&o);
  if (s) return s;
  Topology T;
  T.periodic = (o.flags & AFMM_PERIODIC) != 0;
  s = append_hierarchy(T, *h, 0);
  if (s) return s;
  build_groups(T);
  WorkCounts W;
  if (out) fill_info(*out, W, T, o);
  return AFMM_OK;
}

}  // extern "C"

// Tile records (target level, then `nc` groups = refined ranks at level
// target-1, -1 padded) of one parity class each, appended to `out`; the tiles
// of the 8 classes are interleaved so that a contiguous range of tiles covers
// one region for every class.  Returns the number of tiles appended.
static int append_tiles(const Topology& T, int target, const std::vector<int32_t>& grp, int nc,
                        std::vector<int32_t>& out) {
  std::vector<int32_t> cls[8];
  for (int32_t F : grp) cls[T.lv[target - 1].refcell[F] & 7].push_back(F);
  size_t maxchunks = 0;
  for (auto& c : cls) maxchunks = std::max(maxchunks, (c.size() + nc - 1) / nc);
  int n = 0;
  for (size_t ch = 0; ch < maxchunks; ++ch)
    for (auto& c : cls) {
      if (ch * nc >= c.size()) continue;
      out.push_back(target);
      for (int j = 0; j < nc; ++j) {
        const size_t i = ch * nc + j;
        out.push_back(i < c.size() ? c[i] : -1);
      }
      ++n;
    }
  return n;
}

static void dev_free(afmm_plan* P, void* ptr, size_t bytes) {
  if (!ptr) return;
  for (size_t i = 0; i < P->allocs.size(); ++i)
    if (P->allocs[i].p == ptr) {
      const afmm_plan::Alloc a = P->allocs[i];
      P->allocs.erase(P->allocs.begin() + (long)i);
      if (a.cached) {
        int cur = -1;
        (void)hipGetDevice(&cur);
        if (cur != a.dev) (void)hipSetDevice(a.dev);
        (void)hipDeviceSynchronize();
        if (cur >= 0 && cur != a.dev) (void)hipSetDevice(cur);
        cache_put(a.dev, a.p, a.cap);
      } else {
        (void)hipFree(ptr);
      }
      break;
    }
  P->bytes -= bytes;
}

// Bytes of the partial-sum buffers that the given splits need (the M2P partial
// sets per leaf level, the M2L tap-range partials per FMM level).
static size_t split_buffer_bytes(const afmm_plan* P, const int* m2l_split, const int* m2p_split) {
  const Topology& T = P->topo;
  size_t total = 0;
  for (int l = 3; l <= T.lmax; ++l) {
    if (T.leafgrp[l].empty()) continue;
    const int pr = P->m2p_range[l][0];
    total += (size_t)m2p_split[pr] * T.lv[l - 1].nref() * 32 * (pr ? sizeof(float) : sizeof(double));
  }
  for (int f = 3; f <= T.lmax - 1; ++f) {
    const int pm = P->m2l_range[f][0];
    if (m2l_split[pm] > 1 && P->m2l_range[f][2] > 0)
      total += (size_t)m2l_split[pm] * T.lv[f].nref() * P->K * (pm ? sizeof(float) : sizeof(double));
  }
  return total;
}

// Frees the partial-sum buffers of every level (callers synchronise first).
static void release_split_buffers(afmm_plan* P) {
  for (int l = 0; l <= P->topo.lmax; ++l) {
    LevelDev& D = P->lv[l];
    dev_free(P, D.part, D.part_bytes);
    dev_free(P, D.Lpart, D.Lpart_bytes);
    D.part = D.Lpart = nullptr;
    D.part_bytes = D.Lpart_bytes = 0;
    D.npart = 0;
  }
}

// Allocates the partial-sum buffers for the plan's current splits into lv[];
// on failure frees what it allocated and leaves every level without buffers.
static afmm_status place_split_buffers(afmm_plan* P) {
  const Topology& T = P->topo;
  const int K = P->K;
  afmm_status s = AFMM_OK;
  for (int l = 3; l <= T.lmax && !s; ++l) {
    if (T.leafgrp[l].empty()) continue;
    const int pr = P->m2p_range[l][0];
    const size_t b = (size_t)P->m2p_split[pr] * T.lv[l - 1].nref() * 32 * (pr ? sizeof(float) : sizeof(double));
    void* q = nullptr;
    if ((s = dev_alloc(P, &q, b))) break;
    P->lv[l - 1].part = q;
    P->lv[l - 1].part_bytes = b;
    P->lv[l - 1].npart = P->m2p_split[pr];
  }
  for (int f = 3; f <= T.lmax - 1 && !s; ++f) {
    const int pm = P->m2l_range[f][0];
    if (P->m2l_split[pm] > 1 && P->m2l_range[f][2] > 0) {
      const size_t b = (size_t)P->m2l_split[pm] * T.lv[f].nref() * K * (pm ? sizeof(float) : sizeof(double));
      void* q = nullptr;
      if ((s = dev_alloc(P, &q, b))) break;
      P->lv[f].Lpart = q;
      P->lv[f].Lpart_bytes = b;
    }
  }
  if (s) release_split_buffers(P);
  return s;
}

// Partial-sum buffers for the plan's current splits (m2l_split / m2p_split),
// replacing earlier ones.  The old buffers are released first (after a device
// sync: kernels may still read them), so that a cap on device memory never
// has to hold both sets.  If the new ones cannot be allocated (max_device_bytes
// or hipMalloc) and the caller passes the previous splits, those splits and
// buffers of their size are restored and the error returned: the plan stays
// consistent.  Only if even that fails is the plan marked unusable.  The
// device copy of lv[] is refreshed in every case.
static afmm_status alloc_split_buffers(afmm_plan* P, const int* prev_m2l = nullptr, const int* prev_m2p = nullptr) {
  const bool had = P->d_lvs != nullptr;
  drop_graphs(P);  // captured launches hold the old buffers and grids
  if (had && hipDeviceSynchronize() != hipSuccess) {
    P->dead = true;
    return fail(AFMM_E_DEVICE, "sync before reallocation");
  }
  release_split_buffers(P);
  afmm_status s = place_split_buffers(P);
  if (s) {
    const std::string why = g_last_error;
    if (prev_m2l && prev_m2p) {
      for (int pr = 0; pr < 2; ++pr) {
        P->m2l_split[pr] = prev_m2l[pr];
        P->m2p_split[pr] = prev_m2p[pr];
      }
      if (place_split_buffers(P)) P->dead = true;
    } else if (had) {
      P->dead = true;
    }
    g_last_error = why + (P->dead ? " (the previous buffers could not be restored: plan unusable)" : "");
  }
  if (had && hipMemcpy(P->d_lvs, P->lv, sizeof(LevelDev) * (kMaxLevel + 1), hipMemcpyHostToDevice) != hipSuccess) {
    P->dead = true;
    return fail(AFMM_E_DEVICE, "level table refresh failed");
  }
  return s;
}

static afmm_status adjoint_topology(afmm_plan* P);
static bool adjoint_noalloc_may_fit(const afmm_plan* P);

// Allocate and upload everything of a plan whose topology is built.
static afmm_status plan_finish(afmm_plan* P, hipStream_t st) {
  Topology& T = P->topo;
  const int K = P->K;
  const bool mixed = P->opt.precision == AFMM_FP32_MIXED;
  const int f64 = mixed ? P->opt.fp64_levels : 1 << 20;
  build_groups(T);
  P->tabs = tables_for(P->opt.p);
  afmm_status s;
  for (int l = 0; l <= T.lmax; ++l) {
    HostLevel& H = T.lv[l];
    LevelDev& D = P->lv[l];
    D.n = H.n();
    D.nref = H.nref();
    int32_t *rank, *slot, *refcell, *nbr;
    if ((s = upload(P, H.rank, &rank, st)) || (s = upload(P, H.slot, &slot, st)) ||
        (s = upload(P, H.refcell, &refcell, st)) || (s = upload(P, H.nbr, &nbr, st)))
      return s;
    D.rank = rank;
    D.slot = slot;
    D.refcell = refcell;
    D.nbr = nbr;
    void* p = nullptr;
    if ((s = dev_alloc(P, &p, (size_t)D.n * sizeof(double)))) return s;
    D.mass = (double*)p;
    if ((s = dev_alloc(P, &p, (size_t)D.nref * K * sizeof(double)))) return s;
    D.S64 = (double*)p;
    // source copies: FP32 where an FP32 kernel reads this level (M2L of f = l+1 or
    // M2P of l+1 when l >= f64; near-field M2P of l when l > f64+1), FP64 where an
    // FP64 kernel does (l <= f64 + 1)
    // Each copy has one extra row of zeros after the nref rows: the MFMA tap
    // loops read it for a missing or leaf source, so that their loads need no
    // branch.
    if (mixed && l >= f64) {
      const size_t row = (size_t)src_row(P->opt.p, 4) * sizeof(float);
      if ((s = dev_alloc(P, &p, (size_t)(D.nref + 1) * row))) return s;
      if (hipMemsetAsync((char*)p + (size_t)D.nref * row, 0, row, st) != hipSuccess)
        return fail(AFMM_E_DEVICE, "zero row of the source copy");
      D.S32 = (float*)p;
    }
    if (!mixed || l <= f64 + 1) {
      const size_t row = (size_t)src_row(P->opt.p, 8) * sizeof(double);
      if ((s = dev_alloc(P, &p, (size_t)(D.nref + 1) * row))) return s;
      if (hipMemsetAsync((char*)p + (size_t)D.nref * row, 0, row, st) != hipSuccess)
        return fail(AFMM_E_DEVICE, "zero row of the source copy");
      D.Sc64 = (double*)p;
    }
    if (l <= f64) {
      if ((s = dev_alloc(P, &p, (size_t)D.nref * K * sizeof(double)))) return s;
      D.L64 = (double*)p;
    } else {
      if ((s = dev_alloc(P, &p, (size_t)D.nref * K * sizeof(float)))) return s;
      D.L32 = (float*)p;
    }
  }
  for (int l = 0; l <= T.lmax; ++l) {
    if ((s = upload(P, T.leafgrp[l], &P->d_leafgrp[l], st))) return s;
    if ((s = upload(P, T.m2lgrp[l], &P->d_m2lgrp[l], st))) return s;
    if ((s = upload(P, T.nmgrp[l], &P->d_nmgrp[l], st))) return s;
    if ((s = upload(P, T.adjvgrp[l], &P->d_adjvgrp[l], st))) return s;
    if ((s = upload(P, T.upleaf[l], &P->d_upleaf[l], st))) return s;
    if ((s = upload(P, T.upmix[l], &P->d_upmix[l], st))) return s;
    if (!T.nmgrp[l].empty()) {
      const size_t es = (mixed && (l - 1) > f64) ? sizeof(float) : sizeof(double);
      // groups without refined near candidates are never written: zero once
      const size_t bytes = (size_t)T.lv[l - 1].nref() * 32 * es;
      if ((s = dev_alloc(P, &P->d_nmp[l], bytes))) return s;
      if (hipMemsetAsync(P->d_nmp[l], 0, bytes, st) != hipSuccess) return fail(AFMM_E_DEVICE, "near partial clear");
    }
  }
  const HostTables& H = *P->tabs;
  {
    std::vector<int8_t> mi8(H.mi.begin(), H.mi.end());
    int8_t* d_mi;
    int16_t *d_sum, *d_up, *d_m2p_off, *d_m2l_off;
    double* d_binom;
    int32_t *d_taps, *d_tinfo;
    if ((s = upload(P, mi8, &d_mi, st)) || (s = upload(P, H.sumidx, &d_sum, st)) || (s = upload(P, H.up, &d_up, st)) ||
        (s = upload(P, H.binom, &d_binom, st)) || (s = upload(P, H.taps, &d_taps, st)) ||
        (s = upload(P, H.m2p_off, &d_m2p_off, st)) || (s = upload(P, H.m2l_off, &d_m2l_off, st)) ||
        (s = upload(P, H.m2l_tinfo, &d_tinfo, st)))
      return s;
    P->cm.mi = d_mi;
    P->cm.sumidx = d_sum;
    P->cm.up = d_up;
    P->cm.binom = d_binom;
    // The upward pass writes the source copies c_a 2^|a| S~_a that every
    // translation reads; with the paper's cap (multipoles to order p - 1) the
    // factor of the order-p coefficients is 0, so M2L, M2P and the near-field
    // M2P see them as absent, and the adjoint's transpose of the same scaling
    // drops their bars.
    std::vector<double> c2 = H.cfac2;
    if (P->opt.flags & AFMM_PAPER_QUAD_CAP)
      for (int a = 0; a < K; ++a)
        if (H.mi[4 * a + 3] == P->opt.p) c2[a] = 0.0;
    const double* d_c2 = nullptr;
    if ((s = upload_conv<double>(P, c2, &d_c2, st))) return s;
    P->cm.cfac2 = d_c2;
    int32_t *d_ms, *d_ml;
    double* d_mw;
    if ((s = upload(P, H.m2m_start, &d_ms, st)) || (s = upload(P, H.m2m_list, &d_ml, st)) ||
        (s = upload(P, H.m2m_w, &d_mw, st)))
      return s;
    P->cm.m2m_start = d_ms;
    P->cm.m2m_list = d_ml;
    P->cm.m2m_w = d_mw;
    int32_t *d_ts, *d_tl, *d_tt;
    double* d_tw;
    if ((s = upload(P, H.m2mT_start, &d_ts, st)) || (s = upload(P, H.m2mT_list, &d_tl, st)) ||
        (s = upload(P, H.m2mT_w, &d_tw, st)) || (s = upload(P, H.tapsT, &d_tt, st)))
      return s;
    P->cm.m2mT_start = d_ts;
    P->cm.m2mT_list = d_tl;
    P->cm.m2mT_w = d_tw;
    P->cm.tapsT = d_tt;
    int16_t *d_ap, *d_al;
    if ((s = upload(P, H.adj_m2p_off, &d_ap, st)) || (s = upload(P, H.adj_m2l_off, &d_al, st))) return s;
    P->cm.adj_m2p_off = d_ap;
    P->cm.adj_m2l_off = d_al;
    int32_t *d_lts, *d_ltl;
    double* d_ltw;
    if ((s = upload(P, H.l2lT_start, &d_lts, st)) || (s = upload(P, H.l2lT_list, &d_ltl, st)) ||
        (s = upload(P, H.l2lT_w, &d_ltw, st)))
      return s;
    P->cm.l2lT_start = d_lts;
    P->cm.l2lT_list = d_ltl;
    P->cm.l2lT_w = d_ltw;
    P->mt.taps = d_taps;
    P->mt.m2p_off = d_m2p_off;
    P->mt.m2l_off = d_m2l_off;
    P->mt.m2l_tinfo = d_tinfo;
  }
  // D~ rows in the LDS stage layout of the MFMA kernels (per element type: the
  // padding is to whole 16-byte vectors)
  auto dstage = [&](int bytes) {
    const int p = P->opt.p, ks = dstage_ks(p), len = dstage_len(p, bytes);
    std::vector<double> v((size_t)kNumD * len, 0.0);
    for (int di = 0; di < kNumD; ++di)
      for (int o = 0; o < 8; ++o)
        for (int g = 0; g < K; ++g) v[(size_t)di * len + o * ks + g] = H.Dil[((size_t)di * 8 + o) * K + g];
    return v;
  };
  if ((s = upload_conv<double>(P, dstage(8), &P->t64.Dstage, st))) return s;
  if (mixed && (s = upload_conv<float>(P, dstage(4), &P->t32.Dstage, st))) return s;
  // near-field operator regrouped into 16-byte vectors of consecutive MFMA
  // steps per lane: [t][kb / VW][lane][kb % VW]
  auto near_vec = [&](int bytes) {
    const int NKB = near_ksteps(P->opt.p), vw = 16 / bytes;
    std::vector<double> v(H.nearA.size());
    for (int t = 0; t < 2; ++t)
      for (int kb = 0; kb < NKB; ++kb)
        for (int lane = 0; lane < 64; ++lane)
          v[(((size_t)t * (NKB / vw) + kb / vw) * 64 + lane) * vw + kb % vw] = H.nearA[((size_t)t * NKB + kb) * 64 + lane];
    return v;
  };
  if ((s = upload_conv<double>(P, near_vec(8), &P->t64.nearA, st))) return s;
  // the same-level part transposed, for the adjoint: row op (source child of
  // the column's group, rows 8..15 zero), column 32 e' + 4 o + q: target child
  // o of the group's neighbour e', quantity q (the forward row 8 q + o), whose
  // group sees the source at slot 8 (26 - e') + op
  {
    const int NKB = near_ksteps(P->opt.p);
    auto Aat = [&](int R, int k) { return H.nearA[((size_t)(R >> 4) * NKB + (k >> 2)) * 64 + (R & 15) + 16 * (k & 3)]; };
    std::vector<double> at((size_t)216 * 64, 0.0);
    for (int kb = 0; kb < 216; ++kb)
      for (int lane = 0; lane < 64; ++lane) {
        const int row = lane & 15, kk = 4 * kb + (lane >> 4);
        if (row >= 8) continue;
        const int e = kk >> 5, j = kk & 31, o = j >> 2, q = j & 3;
        at[(size_t)kb * 64 + lane] = Aat(8 * q + o, 8 * (26 - e) + row);
      }
    if ((s = upload_conv<double>(P, at, &P->t64.adjNearA, st))) return s;
  }
  if (mixed && (s = upload_conv<float>(P, near_vec(4), &P->t32.nearA, st))) return s;
  if ((s = upload_conv<double>(P, H.Dsame, &P->t64.Dsame, st)) ||
      (s = upload_conv<double>(P, H.cfac2, &P->t64.cfac2, st)) || (s = upload_conv<double>(P, H.cfacn, &P->t64.cfacn, st)) ||
      (s = upload_conv<double>(P, H.l2lw, &P->t64.l2lw, st)) || (s = upload_conv<double>(P, H.l2p, &P->t64.l2p, st)))
    return s;
  if (mixed) {
    if ((s = upload_conv<float>(P, H.Dsame, &P->t32.Dsame, st)) ||
        (s = upload_conv<float>(P, H.cfac2, &P->t32.cfac2, st)) || (s = upload_conv<float>(P, H.cfacn, &P->t32.cfacn, st)) ||
        (s = upload_conv<float>(P, H.l2lw, &P->t32.l2lw, st)) || (s = upload_conv<float>(P, H.l2p, &P->t32.l2p, st)))
      return s;
  }
  // parity-class tiles of the MFMA kernels (all levels of one precision in one
  // array) and the intermediate-field partials
  {
    std::vector<int32_t> m2p_rec[2], m2l_rec[2], m2p_rec2[2];
    int m2p_nc[2] = {m2p_columns(P->opt.p, false), m2p_columns(P->opt.p, true)};
    // 32-group tiles for tile shape 2, where the order and precision allow it
    const bool two[2] = {m2p_shape_ok(P->opt.p, false, 2), m2p_shape_ok(P->opt.p, true, 2)};
    for (int l = 3; l <= T.lmax; ++l) {
      const int pr = (mixed && (l - 1) > f64) ? 1 : 0;
      const int n0 = (int)(m2p_rec[pr].size() / (m2p_nc[pr] + 1));
      const int n = append_tiles(T, l, T.leafgrp[l], m2p_nc[pr], m2p_rec[pr]);
      P->m2p_range[l][0] = pr;
      P->m2p_range[l][1] = n0;
      P->m2p_range[l][2] = n;
      if (two[pr]) {
        const int c = m2p_shape_columns(2);
        const int q0 = (int)(m2p_rec2[pr].size() / (c + 1));
        P->m2p_range2[l][0] = pr;
        P->m2p_range2[l][1] = q0;
        P->m2p_range2[l][2] = append_tiles(T, l, T.leafgrp[l], c, m2p_rec2[pr]);
      }
      const int pm = (mixed && l > f64) ? 1 : 0;
      if (l <= T.lmax - 1) {
        const int m0 = (int)(m2l_rec[pm].size() / 17);
        const int m = append_tiles(T, l, T.m2lgrp[l], 16, m2l_rec[pm]);
        P->m2l_range[l][0] = pm;
        P->m2l_range[l][1] = m0;
        P->m2l_range[l][2] = m;
      }
    }
    // M2L launches with few tiles split their 189 taps over several blocks
    int ncu = 256;
    {
      int dev = 0;
      if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
      if (ncu <= 0) ncu = 256;
    }
    for (int pr = 0; pr < 2; ++pr) {
      const int nt = (int)(m2l_rec[pr].size() / 17);
      P->m2l_split[pr] = P->opt.tap_split > 0 ? P->opt.tap_split
                         : nt > 0              ? std::max(1, std::min(21, (2 * ncu + nt - 1) / nt))
                                               : 1;
    }
    // M2P likewise, aiming at 12 waves per CU; each tap range writes its own
    // partial set, summed in order by the leaf kernel
    for (int pr = 0; pr < 2; ++pr) {
      const int nt = (int)(m2p_rec[pr].size() / (m2p_nc[pr] + 1));
      P->m2p_split[pr] = P->opt.tap_split > 0 ? P->opt.tap_split
                         : nt > 0              ? std::max(1, std::min(8, (12 * ncu + nt - 1) / nt))
                                               : 1;
    }
    if ((s = alloc_split_buffers(P))) return s;
    for (int pr = 0; pr < 2; ++pr) {
      int32_t* d = nullptr;
      if ((s = upload(P, m2p_rec[pr], &d, st))) return s;
      P->m2p_all[pr] = {d, (int)(m2p_rec[pr].size() / (m2p_nc[pr] + 1)), m2p_nc[pr]};
      if (two[pr] && !m2p_rec2[pr].empty()) {
        if ((s = upload(P, m2p_rec2[pr], &d, st))) return s;
        const int c = m2p_shape_columns(2);
        P->m2p_all2[pr] = {d, (int)(m2p_rec2[pr].size() / (c + 1)), c};
      }
      P->m2p_shape[pr] = m2p_shape_ok(P->opt.p, pr == 1, P->opt.m2p_shape) ? P->opt.m2p_shape : 0;
      if ((s = upload(P, m2l_rec[pr], &d, st))) return s;
      P->m2l_all[pr] = {d, (int)(m2l_rec[pr].size() / 17), 16};
    }
    // ATS chains: walking up from the groups of target level l, the needed
    // cells of FMM level f are the refined ancestors of level-l leaves; the
    // M2L group of f-1 is needed when one of its children is
    for (int l = 4; l <= T.lmax; ++l) {
      if (T.leafgrp[l].empty()) continue;
      auto& A = P->ats[l];
      std::vector<char> need(T.lv[l - 1].nref(), 0);
      for (int32_t F : T.leafgrp[l]) need[F] = 1;
      std::vector<int32_t> grp[kMaxLevel];
      for (int f = l - 1; f >= 3; --f) {
        std::vector<char> up(T.lv[f - 1].nref(), 0);
        for (int32_t G : T.m2lgrp[f]) {
          bool any = false;
          for (int o = 0; o < 8 && !any; ++o) {
            const int32_t rc = T.lv[f].rank[8 * G + o];
            any = rc >= 0 && need[rc];
          }
          if (any) {
            grp[f].push_back(G);
            up[G] = 1;
          }
        }
        need.swap(up);
      }
      std::vector<int32_t> rec[2];
      for (int f = 3; f <= l - 1; ++f) {
        const int pm = P->m2l_range[f][0];
        const int m0 = (int)(rec[pm].size() / 17);
        const int m = append_tiles(T, f, grp[f], 16, rec[pm]);
        A.m2l_range[f][0] = pm;
        A.m2l_range[f][1] = m0;
        A.m2l_range[f][2] = m;
        A.ngrp[f] = (int)grp[f].size();
        if ((s = upload(P, grp[f], &A.d_grp[f], st))) return s;
      }
      for (int pr = 0; pr < 2; ++pr) {
        int32_t* d = nullptr;
        if ((s = upload(P, rec[pr], &d, st))) return s;
        A.m2l_all[pr] = {d, (int)(rec[pr].size() / 17), 16};
      }
      A.on = true;
    }
  }
  {
    std::vector<LevelDev> lvh(P->lv, P->lv + kMaxLevel + 1);
    if ((s = upload(P, lvh, &P->d_lvs, st))) return s;
  }
  void* p = nullptr;
  if ((s = dev_alloc(P, &p, (size_t)std::max<int64_t>(T.nslots, 1) * sizeof(double)))) return s;
  P->m_snap = (double*)p;
  if ((s = dev_alloc(P, &p, sizeof(int)))) return s;
  P->d_flag = (int*)p;
  if (hipHostMalloc((void**)&P->h_flag, sizeof(int), hipHostMallocDefault) != hipSuccess) {
    P->h_flag = nullptr;
    return fail(AFMM_E_OUT_OF_MEMORY, "pinned flag allocation failed");
  }
  P->cself = (P->opt.flags & AFMM_SELF_POTENTIAL) ? cube_self_constant() : 0.0;
  if (T.periodic) {
    const auto tab = periodic_far_table(P->opt.p);
    std::vector<double> cf(K);
    for (int a = 0; a < K; ++a) {
      const int* m = &P->tabs->mi[4 * a];
      cf[a] = ((m[3] & 1) ? -1.0 : 1.0) / (fact(m[0]) * fact(m[1]) * fact(m[2]));
      if ((P->opt.flags & AFMM_PAPER_QUAD_CAP) && m[3] == P->opt.p) cf[a] = 0.0;
    }
    if ((s = upload_conv<double>(P, *tab, &P->d_pfar, st)) || (s = upload_conv<double>(P, cf, &P->d_pfar_cf, st)))
      return s;
    P->l_first = 2;
  }
  // a plan small enough for the allocation-free adjoint gets its adjoint
  // topology now, so that afmm_solve_adjoint_noalloc never has to allocate it
  if (T.levelmin.size() == 1 && adjoint_noalloc_may_fit(P) && (s = adjoint_topology(P))) return s;
  if ((P->opt.flags & AFMM_GRAPH) && hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking) != hipSuccess)
    return fail(AFMM_E_DEVICE, "capture stream creation failed");
  if (hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming) != hipSuccess)
    return fail(AFMM_E_DEVICE, "stream/event creation failed");
  if (hipStreamSynchronize(st) != hipSuccess) return fail(AFMM_E_DEVICE, "upload synchronisation failed");
  return AFMM_OK;
}

// Counts the plan's sizes and work once (the topology is fixed after plan_finish).
static afmm_status ensure_info(const afmm_plan* P) {
  try {
    std::call_once(P->info_once, [P] { fill_info(P->info, P->work, P->topo, P->opt); });
  } catch (const std::bad_alloc&) {
    return fail(AFMM_E_OUT_OF_MEMORY, "host allocation failed while counting the plan's work");
  }
  return AFMM_OK;
}

static afmm_status afmm_plan_create_impl(const afmm_hierarchy* h, const afmm_options* opt, void* hip_stream,
                                        afmm_plan** out) {
  if (!h || !out) return fail(AFMM_E_INVALID_ARG, "null argument");
  *out = nullptr;
  afmm_options o;
  if (opt) o = *opt;
  else afmm_options_default(&o);
  afmm_status s = check_options(&o);
  if (s) return s;
  afmm_plan* P = new afmm_plan();
  try {
    P->opt = o;
    P->K = nmi(o.p);
    P->topo.periodic = (o.flags & AFMM_PERIODIC) != 0;
    s = append_hierarchy(P->topo, *h, 0);
    if (!s) s = plan_finish(P, (hipStream_t)hip_stream);
  } catch (...) {
    free_plan(P);
    delete P;
    throw;
  }
  if (s) {
    free_plan(P);
    delete P;
    return s;
  }
  *out = P;
  return AFMM_OK;
}

// New plan for a hierarchy whose levels below `level` are those of `old`
// (cells, caller order and refined flags): the stale trees of those levels
// keep the masses of their last rebuild (old's snapshot), the trees of levels
// >= level are new and take their masses from the next solve.
static afmm_status afmm_plan_replan_impl(const afmm_plan* old, const afmm_hierarchy* h, int32_t level,
                                        void* hip_stream, afmm_plan** out) {
  if (!old || !h || !out) return fail(AFMM_E_INVALID_ARG, "null argument");
  *out = nullptr;
  if (old->dead) return fail(AFMM_E_DEVICE, "plan is unusable after an earlier device error");
  const Topology& To = old->topo;
  if (To.levelmin.size() != 1) return fail(AFMM_E_INVALID_ARG, "batched plan: no re-plan");
  const int lmin = To.levelmin[0];
  if (h->levelmin != lmin) return fail(AFMM_E_INVALID_ARG, "levelmin differs from the old plan's");
  if (level < lmin + 1 || level > h->levelmax + 1)
    return fail(AFMM_E_INVALID_ARG, "re-planned level must be in [levelmin + 1, levelmax + 1]");
  afmm_plan* P = nullptr;
  afmm_status s = afmm_plan_create_impl(h, &old->opt, hip_stream, &P);
  if (s) return s;
  const Topology& Tn = P->topo;
  bool same = Tn.level_off[0].size() >= (size_t)(level - lmin + 1) &&
              To.level_off[0].size() >= (size_t)(level - lmin + 1) && Tn.lmax >= level - 1 && To.lmax >= level - 1;
  for (int l = 0; same && l <= level - 1; ++l)
    same = Tn.lv[l].rank == To.lv[l].rank && Tn.lv[l].slot == To.lv[l].slot;
  for (int i = 0; same && i <= level - lmin; ++i) same = Tn.level_off[0][i] == To.level_off[0][i];
  if (!same) {
    free_plan(P);
    delete P;
    return fail(AFMM_E_INVALID_ARG, "levels below the re-planned level differ from the old plan's");
  }
  hipStream_t st = (hipStream_t)hip_stream;
  if (old->snap_valid) {
    const size_t n = (size_t)Tn.level_off[0][level - lmin];
    if (n > 0 && (hipMemcpyAsync(P->m_snap, old->m_snap, n * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess ||
                  hipStreamSynchronize(st) != hipSuccess)) {
      free_plan(P);
      delete P;
      return fail(AFMM_E_DEVICE, "snapshot copy failed");
    }
    P->snap_valid = true;
    P->fresh_from = level;
  }
  *out = P;
  return AFMM_OK;
}

extern "C" afmm_status afmm_release_cached_memory(void) {
  cache_release(-1);
  return AFMM_OK;
}

extern "C" afmm_status afmm_plan_destroy(afmm_plan* P) {
  if (!P) return AFMM_OK;
  free_plan(P);
  delete P;
  return AFMM_OK;
}

extern "C" afmm_status afmm_plan_get_info(const afmm_plan* P, afmm_plan_info* out) {
  if (!P || !out) return fail(AFMM_E_INVALID_ARG, "null argument");
  if (afmm_status s = ensure_info(P)) return s;
  *out = P->info;
  out->device_bytes = P->bytes;  // live: the autotuner and the adjoint change it
  return AFMM_OK;
}

// ---------------------------------------------------------------------------
// solve driver

// AFMM_CHECK_INPUT: flag any non-finite mass among the leaf slots of one level
__global__ void k_nonfinite(int n, const int32_t* __restrict__ rank, const int32_t* __restrict__ slot,
                            const double* __restrict__ m, int* __restrict__ flag) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int s = slot[i];
    if (rank[i] < 0 && s >= 0 && !isfinite(m[s])) flag[0] = 1;
  }
}
__global__ void k_flag_clear(int* __restrict__ flag) { flag[0] = 0; }

static afmm_status dev_check(afmm_plan* P, hipError_t e, const char* what) {
  if (e == hipSuccess) return AFMM_OK;
  P->dead = true;
  return fail(AFMM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// ---- per-launch event timing ----
enum { kGather = 0, kUpward, kM2L64, kM2L32, kL2L, kM2P64, kM2P32, kLeaf64, kLeaf32,
       kAdjNear, kAdjM2P, kAdjM2L, kAdjTree, kNumKinds };
static const char* kKindName[kNumKinds] = {"gather", "upward", "m2l_f64", "m2l_f32", "l2l",
                                           "m2p_f64", "m2p_f32", "near_f64", "near_f32",
                                           "adj_near", "adj_m2p", "adj_m2l", "adj_tree"};

static hipEvent_t pool_get(afmm_plan* P) {
  if (!P->event_pool.empty()) {
    hipEvent_t e = P->event_pool.back();
    P->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

static hipEvent_t prof_begin(afmm_plan* P, hipStream_t st) {
  if (!P->profiling) return nullptr;
  hipEvent_t a = pool_get(P);
  if (a) (void)hipEventRecord(a, st);
  return a;
}

static void prof_end(afmm_plan* P, hipEvent_t a, hipStream_t st, int kind, int level) {
  if (!P->profiling || !a) return;
  hipEvent_t b = pool_get(P);
  if (!b) return;
  (void)hipEventRecord(b, st);
  P->recs.push_back({kind, level, a, b, P->pending_flops, P->pending_bytes});
  P->pending_flops = P->pending_bytes = 0.0;
}

// Upward pass over every level, M2L over FMM levels 3..fmax, leaf evaluation
// for the levels in [lo, hi].  Masses come from `msrc` (slot space); with
// `snap`, the mass gather also copies every slot there.
static afmm_status run_solve(afmm_plan* P, const double* msrc, int fmax, int lo, int hi, double* phi, double* acc,
                             hipStream_t st, bool keep_trees = false, double* snap = nullptr) {
  Topology& T = P->topo;
  const int p = P->opt.p;
  const bool mixed = P->opt.precision == AFMM_FP32_MIXED;
  const int f64 = mixed ? P->opt.fp64_levels : 1 << 20;
  afmm_status s;
  // keep_trees: the level masses and multipoles on the device already belong to msrc
  for (int l = T.lmin_all; l <= T.lmax && !keep_trees; ++l) {
    hipEvent_t a = prof_begin(P, st);
    if ((s = dev_check(P, launch_gather_mass(P->lv[l], msrc, snap, st), "gather"))) return s;
    prof_end(P, a, st, kGather, l);
  }
  for (int f = T.lmax - 1; f >= 2 && !keep_trees; --f) {
    hipEvent_t a = prof_begin(P, st);
    if ((s = dev_check(P,
                       launch_upward(p, P->d_upleaf[f], (int)T.upleaf[f].size(), P->d_upmix[f],
                                     (int)T.upmix[f].size(), P->lv[f], P->lv[f + 1], P->cm, st),
                       "upward")))
      return s;
    prof_end(P, a, st, kUpward, f);
  }
  // periodic boxes: local expansions of the 64 level-2 cells from the far operator
  if (T.periodic) {
    hipEvent_t a = prof_begin(P, st);
    if ((s = dev_check(P, launch_periodic_far(p, P->lv[2], P->d_pfar, P->d_pfar_cf, P->cm, st), "periodic far")))
      return s;
    prof_end(P, a, st, kL2L, 2);
  }
  // fork: the intermediate field (M2P, one large launch) runs on the side
  // stream while the downward chain (M2L taps, then the latency-bound L2L
  // levels) runs on this one; the chain is enqueued without a wait, so its
  // small first launches get the CUs first and M2P fills the rest.  Serial
  // plans (and profiled solves: events then time one launch at a time) use
  // one stream.
  const bool serial = !(P->opt.flags & AFMM_OVERLAP) || (P->opt.flags & AFMM_SERIAL) || P->profiling || P->capturing;
  hipStream_t sm = serial ? st : P->side;
  if (!serial && ((s = dev_check(P, hipEventRecord(P->ev_fork, st), "fork")) ||
                  (s = dev_check(P, hipStreamWaitEvent(sm, P->ev_fork, 0), "fork"))))
    return s;
  // intermediate field (M2P) of the leaf levels lo..hi: one launch per precision
  for (int pr = 0; pr < 2; ++pr) {
    const int shape = P->m2p_shape[pr];
    const int(*range)[3] = shape == 2 ? P->m2p_range2 : P->m2p_range;
    int t0 = -1, n = 0;
    for (int l = std::max(lo, 3); l <= hi; ++l)
      if (P->m2p_range[l][0] == pr && range[l][2] > 0) {
        if (t0 < 0) t0 = range[l][1];
        n = range[l][1] + range[l][2] - t0;
      }
    if (n <= 0) continue;
    hipEvent_t a = prof_begin(P, sm);
    if ((s = dev_check(P, launch_m2p(p, pr == 1, shape == 2 ? P->m2p_all2[pr] : P->m2p_all[pr], t0, n,
                                     P->m2p_split[pr], shape, P->mt, P->d_lvs, P->t32, P->t64, sm), "m2p")))
      return s;
    for (int l = std::max(lo, 3); l <= hi; ++l)
      if (P->m2p_range[l][0] == pr) {
        P->pending_flops += P->work.m2p_flops[l];
        P->pending_bytes += P->work.m2p_bytes[l];
      }
    prof_end(P, a, sm, pr ? kM2P32 : kM2P64, -1);
  }
  if (!serial && (s = dev_check(P, hipEventRecord(P->ev_join, sm), "join"))) return s;
  // M2L tap sums of FMM levels 3..fmax: one launch per precision.  A solve of
  // one target level takes its ATS chain (ancestors of the level's leaves only).
  const afmm_plan::AtsChain* chain = (lo == hi && P->ats[lo].on) ? &P->ats[lo] : nullptr;
  const MfmaTiles* m2l_all = chain ? chain->m2l_all : P->m2l_all;
  const int(*m2l_range)[3] = chain ? chain->m2l_range : P->m2l_range;
  for (int pr = 0; pr < 2; ++pr) {
    int t0 = -1, n = 0;
    for (int f = 3; f <= fmax; ++f)
      if (m2l_range[f][0] == pr && m2l_range[f][2] > 0) {
        if (t0 < 0) t0 = m2l_range[f][1];
        n = m2l_range[f][1] + m2l_range[f][2] - t0;
      }
    if (n <= 0) continue;
    hipEvent_t a = prof_begin(P, st);
    if ((s = dev_check(P, launch_m2l_taps(p, pr == 1, m2l_all[pr], t0, n, P->m2l_split[pr], P->mt, P->d_lvs,
                                          P->t32, P->t64, st),
                       "m2l")))
      return s;
    for (int f = 3; f <= fmax; ++f)
      if (m2l_range[f][0] == pr && m2l_range[f][2] > 0) {
        const double frac = chain ? (double)chain->ngrp[f] / (double)std::max<size_t>(T.m2lgrp[f].size(), 1) : 1.0;
        P->pending_flops += frac * P->work.m2l_flops[f];
        P->pending_bytes += frac * P->work.m2l_bytes[f];
      }
    prof_end(P, a, st, pr ? kM2L32 : kM2L64, -1);
  }
  // completion of each FMM level: tap-range partials (if split) + ShiftLocal (L2L) of the father
  for (int f = 3; f <= fmax; ++f) {
    const int ng = chain ? chain->ngrp[f] : (int)T.m2lgrp[f].size();
    const int32_t* grp = chain ? chain->d_grp[f] : P->d_m2lgrp[f];
    const int ns = P->m2l_split[P->m2l_range[f][0]];
    if (ng == 0 || (f - 1 < P->l_first && ns == 1)) continue;
    hipEvent_t a = prof_begin(P, st);
    if ((s = dev_check(P,
                       launch_l2l(p, mixed && f > f64, mixed && (f - 1) > f64, f - 1 >= P->l_first, ns, grp, ng,
                                  P->lv[f - 1], P->lv[f], P->t32, P->t64, P->cm, st),
                       "l2l")))
      return s;
    prof_end(P, a, st, kL2L, f);
  }
  // join: the leaf kernel needs the intermediate-field partials
  if (!serial && (s = dev_check(P, hipStreamWaitEvent(st, P->ev_join, 0), "join"))) return s;
  // far, near and nearest fields + output, per leaf level
  for (int l = std::max(lo, 1); l <= hi; ++l) {
    const int ng = (int)T.leafgrp[l].size();
    if (ng == 0) continue;
    const LevelDev empty;
    const LevelDev& lvp = l + 1 <= T.lmax ? P->lv[l + 1] : empty;
    const double h = P->opt.boxlen / (double)(1LL << l);
    const bool fp32 = mixed && (l - 1) > f64;
    hipEvent_t a = prof_begin(P, st);
    const int nm = (int)T.nmgrp[l].size();
    if (nm > 0 && (s = dev_check(P,
                                 launch_near_m2p(p, fp32, P->d_nmgrp[l], nm, P->lv[l - 1], P->lv[l], lvp, P->t32,
                                                 P->t64, P->d_nmp[l], st),
                                 "near m2p")))
      return s;
    if ((s = dev_check(P,
                       launch_near(p, fp32, l, P->l_first, P->d_leafgrp[l], ng, P->lv[l - 1], P->lv[l], lvp, P->t32,
                                   P->t64, P->cm,
                                   l >= 3 ? P->lv[l - 1].part : nullptr, nm > 0 ? P->d_nmp[l] : nullptr, P->opt.G,
                                   h, P->cself, phi, acc, st),
                       "near")))
      return s;
    prof_end(P, a, st, fp32 ? kLeaf32 : kLeaf64, l);
  }
  return AFMM_OK;
}

// Runs `body` (the launches of one solve, enqueued on the stream it is given)
// on `st`, or with AFMM_GRAPH replays it from a graph captured on first use for
// this key.  Profiled solves always run eagerly (their events time each launch).
template <typename Body>
static afmm_status replay_or_run(afmm_plan* P, int level, bool rebuild, bool keep, const double* m, double* phi,
                                 double* acc, hipStream_t st, Body body) {
  if (!(P->opt.flags & AFMM_GRAPH) || P->profiling) return body(st);
  afmm_plan::GraphEntry* hit = nullptr;
  for (auto& e : P->graphs)
    if (e.level == level && e.rebuild == rebuild && e.keep == keep && e.m == m && e.phi == phi && e.acc == acc)
      hit = &e;
  if (!hit) {
    constexpr size_t kMaxGraphs = 32;
    if (P->graphs.size() >= kMaxGraphs) {  // evict the least recently used
      size_t old = 0;
      for (size_t i = 1; i < P->graphs.size(); ++i)
        if (P->graphs[i].used < P->graphs[old].used) old = i;
      if (hipStreamSynchronize(st) != hipSuccess) return dev_check(P, hipGetLastError(), "graph eviction");
      (void)hipGraphExecDestroy(P->graphs[old].x);
      (void)hipGraphDestroy(P->graphs[old].g);
      P->graphs.erase(P->graphs.begin() + (long)old);
    }
    afmm_plan::GraphEntry e{level, rebuild, keep, m, phi, acc, nullptr, nullptr, 0};
    if (hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return dev_check(P, hipGetLastError(), "graph capture begin");
    P->capturing = true;
    afmm_status r = body(P->cap);
    P->capturing = false;
    const hipError_t ee = hipStreamEndCapture(P->cap, &e.g);
    if (r) {
      if (e.g) (void)hipGraphDestroy(e.g);
      return r;
    }
    if (ee != hipSuccess || !e.g) return dev_check(P, ee != hipSuccess ? ee : hipErrorUnknown, "graph capture");
    const hipError_t ei = hipGraphInstantiate(&e.x, e.g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      (void)hipGraphDestroy(e.g);
      return dev_check(P, ei, "graph instantiation");
    }
    P->graphs.push_back(e);
    hit = &P->graphs.back();
  }
  hit->used = ++P->graph_tick;
  return dev_check(P, hipGraphLaunch(hit->x, st), "graph launch");
}

// Drifted solves: the rate snapshot and the drifted-mass buffer, allocated by
// the first drifted solve of a plan (the rates start at zero).
static afmm_status ensure_drift_buffers(afmm_plan* P, hipStream_t st) {
  if (P->rate_snap) return AFMM_OK;
  const size_t n = (size_t)std::max<int64_t>(P->topo.nslots, 1);
  void* a = nullptr;
  void* b = nullptr;
  afmm_status s;
  if ((s = dev_alloc(P, &a, n * sizeof(double))) || (s = dev_alloc(P, &b, n * sizeof(double)))) return s;
  if ((s = dev_check(P, launch_adj_zero((double*)a, n, st), "drift buffers"))) return s;
  P->rate_snap = (double*)a;
  P->m_drift = (double*)b;
  return AFMM_OK;
}

// Trees of levels >= from rebuilt at `time`: record their mass rates (a plain
// solve, d_rate null, records none).
static afmm_status record_rates(afmm_plan* P, const double* d_rate, int from, double time, hipStream_t st) {
  const Topology& T = P->topo;
  const int lmin = T.levelmin[0], lmax = T.levelmax[0];
  if (!d_rate) {
    for (int l = from; l <= lmax; ++l) P->rate_valid[l] = false;
    return AFMM_OK;
  }
  afmm_status s = ensure_drift_buffers(P, st);
  if (s) return s;
  const int64_t off = T.level_off[0][from - lmin];
  if ((s = dev_check(P,
                     hipMemcpyAsync(P->rate_snap + off, d_rate + off, (size_t)(T.nslots - off) * sizeof(double),
                                    hipMemcpyDeviceToDevice, st),
                     "rate snapshot")))
    return s;
  for (int l = from; l <= lmax; ++l) {
    P->rate_valid[l] = true;
    P->t_snap[l] = time;
  }
  return AFMM_OK;
}

// d_rate != nullptr: a drifted solve (afmm_solve_drift) at `time`
static afmm_status afmm_solve_impl(afmm_plan* P, int32_t level, int32_t icount, const double* d_mass, double* d_phi,
                                  double* d_acc, void* hip_stream, double time = 0.0,
                                  const double* d_rate = nullptr) {
  if (!P || !d_mass || !d_phi || !d_acc) return fail(AFMM_E_INVALID_ARG, "null argument");
  if (d_rate && !std::isfinite(time)) return fail(AFMM_E_INVALID_ARG, "time must be finite");
  if (P->dead) return fail(AFMM_E_DEVICE, "plan is unusable after an earlier device error");
  hipStream_t st = (hipStream_t)hip_stream;
  Topology& T = P->topo;
  if (T.levelmin.size() != 1) return fail(AFMM_E_INVALID_ARG, "batched plan: use afmm_batch_solve");
  const int lmin = T.levelmin[0], lmax = T.levelmax[0];
  if (level != AFMM_ALL_LEVELS && (level < lmin || level > lmax))
    return fail(AFMM_E_INVALID_ARG, "level outside [levelmin, levelmax]");
  if (level != AFMM_ALL_LEVELS && icount < 1) return fail(AFMM_E_INVALID_ARG, "icount must be >= 1");
  if (P->opt.flags & AFMM_CHECK_INPUT) {
    // the masses this call reads: every level for a full solve, levels >= level
    // when Alg. 1 rebuilds trees, the re-planned levels after a re-plan, none otherwise
    const bool alg = level == AFMM_ALL_LEVELS || level == lmin || icount > 1;
    const bool reads = alg || P->fresh_from <= lmax;
    const int l0 = level == AFMM_ALL_LEVELS ? lmin : std::min(alg ? level : lmax + 1, P->fresh_from);
    if (reads) {
      afmm_status r;
      hipLaunchKernelGGL(k_flag_clear, dim3(1), dim3(1), 0, st, P->d_flag);
      if ((r = dev_check(P, hipGetLastError(), "input check"))) return r;
      for (int l = l0; l <= lmax; ++l) {
        const LevelDev& D = P->lv[l];
        if (D.n == 0) continue;
        hipLaunchKernelGGL(k_nonfinite, dim3((unsigned)std::min((D.n + 255) / 256, 2048)), dim3(256), 0, st, D.n,
                           D.rank, D.slot, d_mass, P->d_flag);
        if ((r = dev_check(P, hipGetLastError(), "input check"))) return r;
        if (d_rate) {
          hipLaunchKernelGGL(k_nonfinite, dim3((unsigned)std::min((D.n + 255) / 256, 2048)), dim3(256), 0, st, D.n,
                             D.rank, D.slot, d_rate, P->d_flag);
          if ((r = dev_check(P, hipGetLastError(), "input check"))) return r;
        }
      }
      if ((r = dev_check(P, hipMemcpyAsync(P->h_flag, P->d_flag, sizeof(int), hipMemcpyDeviceToHost, st),
                         "input check")) ||
          (r = dev_check(P, hipStreamSynchronize(st), "input check")))
        return r;
      if (*P->h_flag) return fail(AFMM_E_NONFINITE, "non-finite mass (or mass rate) in a leaf slot that the solve reads");
    }
  }
  if (level == AFMM_ALL_LEVELS) {
    // the snapshot is written by the mass gather of this solve
    P->fresh_from = 1 << 20;
    P->snap_valid = true;
    P->solved = true;
    P->last_level = AFMM_ALL_LEVELS;
    P->last_fresh = 0;
    P->tree_fresh = false;
    afmm_status r = replay_or_run(P, AFMM_ALL_LEVELS, true, false, d_mass, d_phi, d_acc, st, [&](hipStream_t s) {
      return run_solve(P, d_mass, T.lmax - 1, lmin, lmax, d_phi, d_acc, s, false, P->m_snap);
    });
    P->tree_fresh = r == AFMM_OK;
    if (r == AFMM_OK) r = record_rates(P, d_rate, lmin, time, st);
    return r;
  }
  // Alg. 1: rebuild trees j >= level iff level == levelmin or icount > 1; after
  // a re-plan the trees of the re-planned levels are new and take this call's masses
  const bool rebuild = (level == lmin) || (icount > 1) || P->fresh_from <= T.lmax;
  if (!P->snap_valid && level != lmin)
    return fail(AFMM_E_ATS_ORDER, "solve(l > levelmin) before any tree was built (call solve(levelmin) first)");
  const int from = std::min((level == lmin) || (icount > 1) ? level : T.lmax + 1, P->fresh_from);
  if (rebuild) P->snap_valid = true;
  P->fresh_from = 1 << 20;
  P->solved = true;
  P->last_level = level;
  P->last_fresh = rebuild ? from : T.lmax + 1;
  // Alg. 1 without a rebuild leaves every tree as it was: the snapshot, hence
  // the level masses and merged multipoles of the previous solve, still hold
  const bool keep = !rebuild && P->tree_fresh;
  P->tree_fresh = false;
  const int64_t off = rebuild ? T.level_off[0][from - lmin] : 0;
  if (d_rate) {
    // drifted solve (eager): rebuilt levels record masses, rates and time; the
    // solve reads the snapshot with every stale level advanced to `time`
    afmm_status r = ensure_drift_buffers(P, st);
    if (!r && rebuild && dev_check(P,
                                   hipMemcpyAsync(P->m_snap + off, d_mass + off,
                                                  (size_t)(T.nslots - off) * sizeof(double), hipMemcpyDeviceToDevice, st),
                                   "snapshot"))
      r = AFMM_E_DEVICE;
    if (!r && rebuild) r = record_rates(P, d_rate, from, time, st);
    if (!r) {
      DriftLevels dl{};
      dl.n = lmax - lmin + 1;
      for (int i = 0; i < dl.n; ++i) {
        const int l = lmin + i;
        dl.off[i] = T.level_off[0][i];
        dl.dt[i] = (P->rate_valid[l] && l < from) ? time - P->t_snap[l] : 0.0;
      }
      dl.off[dl.n] = T.level_off[0][dl.n];
      r = dev_check(P, launch_drift(dl, P->m_snap, P->rate_snap, P->m_drift, T.nslots, st), "drift");
    }
    if (!r) r = run_solve(P, P->m_drift, level - 1, level, level, d_phi, d_acc, st, false);
    return r;
  }
  // a plain rebuild leaves no rates for its levels
  if (rebuild)
    for (int l = from; l <= lmax; ++l) P->rate_valid[l] = false;
  afmm_status r = replay_or_run(P, level + 64 * from, rebuild, keep, d_mass, d_phi, d_acc, st, [&](hipStream_t s) -> afmm_status {
    // the rebuilt trees take the masses of levels >= level from this call
    if (rebuild && dev_check(P,
                             hipMemcpyAsync(P->m_snap + off, d_mass + off, (size_t)(T.nslots - off) * sizeof(double),
                                            hipMemcpyDeviceToDevice, s),
                             "snapshot"))
      return AFMM_E_DEVICE;
    return run_solve(P, P->m_snap, level - 1, level, level, d_phi, d_acc, s, keep);
  });
  P->tree_fresh = r == AFMM_OK;
  return r;
}

extern "C" afmm_status afmm_plan_set_profiling(afmm_plan* P, int32_t enable) {
  if (!P) return fail(AFMM_E_INVALID_ARG, "null plan");
  // timed launches take their flops and bytes from the work counts
  if (afmm_status s = enable ? ensure_info(P) : AFMM_OK) return s;
  P->profiling = enable != 0;
  return AFMM_OK;
}

static afmm_status afmm_plan_get_profile_impl(afmm_plan* P, afmm_stage_time* out, int32_t cap, int32_t* n_out) {
  if (!P || !n_out || (cap > 0 && !out)) return fail(AFMM_E_INVALID_ARG, "null argument");
  afmm_stage_time acc[kNumKinds];
  std::memset(acc, 0, sizeof acc);
  for (int k = 0; k < kNumKinds; ++k) std::snprintf(acc[k].name, sizeof acc[k].name, "%s", kKindName[k]);
  for (auto& r : P->recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return dev_check(P, hipGetLastError(), "profile sync");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    afmm_stage_time& t = acc[r.kind];
    t.launches += 1;
    t.ms += ms;
    const WorkCounts& W = P->work;
    switch (r.kind) {
      case kUpward: t.flops += W.up_flops[r.level]; t.bytes += W.up_bytes[r.level]; break;
      case kM2L64: case kM2L32: t.flops += r.flops; t.bytes += r.bytes; break;
      case kL2L: t.flops += W.l2l_flops[r.level]; t.bytes += W.l2l_bytes[r.level]; break;
      case kM2P64: case kM2P32: t.flops += r.flops; t.bytes += r.bytes; break;
      case kLeaf64: case kLeaf32: t.flops += W.leaf_flops[r.level]; t.bytes += W.leaf_bytes[r.level]; break;
      case kAdjNear: case kAdjM2P: case kAdjM2L: case kAdjTree: t.flops += r.flops; t.bytes += r.bytes; break;
      default: t.bytes += 12.0 * P->lv[r.level].n; break;
    }
    P->event_pool.push_back(r.a);
    P->event_pool.push_back(r.b);
  }
  P->recs.clear();
  int32_t n = 0;
  for (int k = 0; k < kNumKinds; ++k)
    if (acc[k].launches) {
      if (n < cap) out[n] = acc[k];
      ++n;
    }
  *n_out = n;
  return AFMM_OK;
}

static afmm_status capture_batch(afmm_batch* B);
static afmm_status batch_pointer_table(afmm_batch* B, const double* const* d_mass, double* const* d_phi,
                                       double* const* d_acc, hipStream_t st);

// ---------------------------------------------------------------------------
// Autotuner: the tap splits of M2L and M2P set the work per block (how many of
// a tile's 189 source offsets one block sums).  Each candidate is timed with
// per-launch events over a few solves of the caller's data; per precision the
// split with the smallest time of its kernel family plus the family that sums
// its partials (L2L for M2L, the leaf kernel for M2P) is kept.
namespace {
// Restores the plan's profiling switch on every exit path.
struct ProfilingScope {
  afmm_plan* P;
  bool saved;
  ProfilingScope(afmm_plan* p, bool on) : P(p), saved(p->profiling) { P->profiling = on; }
  ~ProfilingScope() { P->profiling = saved; }
};

template <typename SolveFn>
afmm_status autotune_core(afmm_plan* P, SolveFn solve, hipStream_t st, afmm_tune_result* out) {
  ProfilingScope scope(P, true);
  // a candidate whose partial buffers would not fit under max_device_bytes is
  // skipped (its buffers would replace the current ones, so only the growth counts)
  auto fits = [&]() {
    if (!P->opt.max_device_bytes) return true;
    const size_t cur = P->bytes - [&] {
      size_t b = 0;
      for (int l = 0; l <= P->topo.lmax; ++l) b += P->lv[l].part_bytes + P->lv[l].Lpart_bytes;
      return b;
    }();
    return cur + split_buffer_bytes(P, P->m2l_split, P->m2p_split) <= P->opt.max_device_bytes;
  };
  // one warm-up solve and kTimed timed ones; each kind's time is its minimum
  // over the timed solves (robust to a solve slowed by something else on the
  // device, where a mean let 1-2% noise decide between candidates)
  constexpr int kTimed = 5;
  auto measure = [&](double* kind_ms) -> afmm_status {
    afmm_status s;
    for (int r = 0; r < 1 + kTimed; ++r)
      if ((s = solve())) return s;
    if (hipStreamSynchronize(st) != hipSuccess) return fail(AFMM_E_DEVICE, "autotune sync");
    const size_t per = P->recs.size() / (1 + kTimed);
    double cur[kNumKinds];
    for (int k = 0; k < kNumKinds; ++k) kind_ms[k] = per ? 1e300 : 0.0;
    for (size_t i = 0; i < P->recs.size(); ++i) {
      if (i % per == 0) std::memset(cur, 0, sizeof(cur));
      auto& r = P->recs[i];
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, r.a, r.b);
      cur[r.kind] += ms;
      if (i % per == per - 1 && i >= per)
        for (int k = 0; k < kNumKinds; ++k) kind_ms[k] = std::min(kind_ms[k], cur[k]);
      P->event_pool.push_back(r.a);
      P->event_pool.push_back(r.b);
    }
    P->recs.clear();
    return AFMM_OK;
  };
  afmm_status s;
  double k0[kNumKinds];
  // baseline with the current splits
  for (auto& r : P->recs) {
    P->event_pool.push_back(r.a);
    P->event_pool.push_back(r.b);
  }
  P->recs.clear();
  if ((s = measure(k0))) return s;
  double before = 0;
  for (int k = 0; k < kNumKinds; ++k) before += k0[k];
  static const int cand_m2l[] = {1, 2, 3, 4, 6, 8, 12, 16, 21};
  static const int cand_m2p[] = {1, 2, 3, 4, 6, 8};
  // One precision at a time (FP32 first), the other held at its current
  // split: the L2L and leaf kernels sum the partials of both precisions, so a
  // joint sweep would let the larger launch decide the smaller one's split.
  int ncand = 0;
  // `have` = the splits the live partial buffers were allocated for.  The
  // kernels only run (in measure) right after a successful allocation, when
  // the plan's splits equal `have`; a refused allocation puts them back.
  int have_l[2] = {P->m2l_split[0], P->m2l_split[1]}, have_p[2] = {P->m2p_split[0], P->m2p_split[1]};
  auto realloc = [&]() -> afmm_status {
    afmm_status r = alloc_split_buffers(P, have_l, have_p);
    if (r == AFMM_OK)
      for (int q = 0; q < 2; ++q) have_l[q] = P->m2l_split[q], have_p[q] = P->m2p_split[q];
    return r;
  };
  // One candidate: skipped when its buffers would exceed max_device_bytes or
  // hipMalloc refuses them (the previous buffers then stand), else timed; the
  // cost is the split kernel's family plus the family that sums its partials.
  auto trial = [&](int* split, int pr, int c, double& best, int& arg, int kind_a, int kind_b) -> afmm_status {
    const int prev = split[pr];
    split[pr] = c;
    if (!fits()) {
      split[pr] = prev;
      return AFMM_OK;
    }
    afmm_status r = realloc();
    if (r == AFMM_E_OUT_OF_MEMORY && !P->dead) {
      split[pr] = prev;  // the previous splits and buffers were restored
      return AFMM_OK;
    }
    if (r) return r;
    double km[kNumKinds];
    if ((r = measure(km))) return r;
    ++ncand;
    const double t = km[kind_a] + km[kind_b];
    if (t < best) best = t, arg = c;
    return AFMM_OK;
  };
  for (int pr = 1; pr >= 0; --pr) {
    if (P->m2l_all[pr].ntiles == 0) continue;
    double best = 1e300;
    int arg = P->m2l_split[pr];
    for (int c : cand_m2l)
      if ((s = trial(P->m2l_split, pr, c, best, arg, pr ? kM2L32 : kM2L64, kL2L))) return s;
    P->m2l_split[pr] = arg;
  }
  constexpr int kShapes = 4;
  for (int pr = 1; pr >= 0; --pr) {
    if (P->m2p_all[pr].ntiles == 0) continue;
    const int ka = pr ? kM2P32 : kM2P64, kb = pr ? kLeaf32 : kLeaf64;
    double sbest[kShapes];
    int ssplit[kShapes];
    for (int shape = 0; shape < kShapes; ++shape) {
      sbest[shape] = 1e300;
      ssplit[shape] = P->m2p_split[pr];
      if (!m2p_shape_ok(P->opt.p, pr == 1, shape) || (shape == 2 && P->m2p_all2[pr].ntiles == 0)) continue;
      P->m2p_shape[pr] = shape;
      for (int c : cand_m2p)
        if ((s = trial(P->m2p_split, pr, c, sbest[shape], ssplit[shape], ka, kb))) return s;
    }
    // the two fastest shapes at their best splits, timed again in turn three
    // times each: a sweep takes seconds, over which the clocks drift enough
    // to decide a close call between shapes timed early and late
    int sa = -1, sb = -1;
    for (int shape = 0; shape < kShapes; ++shape) {
      if (sbest[shape] >= 1e300) continue;
      if (sa < 0 || sbest[shape] < sbest[sa]) sb = sa, sa = shape;
      else if (sb < 0 || sbest[shape] < sbest[sb]) sb = shape;
    }
    if (sa < 0) continue;
    if (sb >= 0) {
      double tot[2] = {0, 0};
      bool ok = true;  // a refused allocation keeps the sweep's choice
      for (int r = 0; r < 3 && ok; ++r)
        for (int j = 0; j < 2 && ok; ++j) {
          const int shape = j ? sb : sa;
          P->m2p_shape[pr] = shape;
          P->m2p_split[pr] = ssplit[shape];
          const afmm_status q = realloc();
          if (q == AFMM_E_OUT_OF_MEMORY && !P->dead) {
            ok = false;
            break;
          }
          if (q) return q;
          double km[kNumKinds];
          if ((s = measure(km))) return s;
          tot[j] += km[ka] + km[kb];
        }
      if (ok && tot[1] < tot[0]) sa = sb;
    }
    P->m2p_shape[pr] = sa;
    P->m2p_split[pr] = ssplit[sa];
  }
  // the chosen splits were timed, so they fitted then; a refusal now leaves
  // the last timed candidate's splits and buffers (consistent, just not the best)
  if ((s = realloc()) && (s != AFMM_E_OUT_OF_MEMORY || P->dead)) return s;
  double k1[kNumKinds];
  if ((s = measure(k1))) return s;
  double after = 0;
  for (int k = 0; k < kNumKinds; ++k) after += k1[k];
  if (out) {
    for (int pr = 0; pr < 2; ++pr) {
      out->m2l_split[pr] = P->m2l_split[pr];
      out->m2p_split[pr] = P->m2p_split[pr];
      out->m2p_shape[pr] = P->m2p_shape[pr];
    }
    out->ms_before = before;
    out->ms_after = after;
    out->candidates = ncand;
  }
  return AFMM_OK;
}
}  // namespace

static afmm_status afmm_plan_autotune_impl(afmm_plan* P, const double* d_mass, double* d_phi, double* d_acc,
                                          void* hip_stream, afmm_tune_result* out) {
  if (!P || !d_mass || !d_phi || !d_acc) return fail(AFMM_E_INVALID_ARG, "null argument");
  if (P->dead) return fail(AFMM_E_DEVICE, "plan is unusable after an earlier device error");
  const Topology& T = P->topo;
  if (T.levelmin.size() != 1) return fail(AFMM_E_INVALID_ARG, "batched plan: use afmm_batch_autotune");
  hipStream_t st = (hipStream_t)hip_stream;
  const int lmin = T.levelmin[0], lmax = T.levelmax[0];
  auto solve = [&]() { return run_solve(P, d_mass, T.lmax - 1, lmin, lmax, d_phi, d_acc, st); };
  P->tree_fresh = false;  // the candidates' solves rebuild the trees from d_mass
  afmm_status s = autotune_core(P, solve, st, out);
  if (s) return s;
  // the autotune solves were synchronous full solves: they also rebuilt every tree
  if (hipMemcpyAsync(P->m_snap, d_mass, (size_t)T.nslots * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess)
    return dev_check(P, hipGetLastError(), "snapshot");
  P->snap_valid = true;
  P->fresh_from = 1 << 20;
  P->tree_fresh = true;
  P->solved = true;
  P->last_level = AFMM_ALL_LEVELS;
  P->last_fresh = 0;
  return AFMM_OK;
}

static afmm_status afmm_batch_autotune_impl(afmm_batch* B, const double* const* d_mass, double* const* d_phi,
                                           double* const* d_acc, void* hip_stream, afmm_tune_result* out) {
  if (!B || !d_mass || !d_phi || !d_acc) return fail(AFMM_E_INVALID_ARG, "null argument");
  afmm_plan* P = B->plan;
  if (P->dead) return fail(AFMM_E_DEVICE, "batch is unusable after an earlier device error");
  hipStream_t st = (hipStream_t)hip_stream;
  afmm_status s;
  if ((s = batch_pointer_table(B, d_mass, d_phi, d_acc, st))) return s;
  const Topology& T = P->topo;
  auto solve = [&]() -> afmm_status {
    afmm_status r;
    if ((r = dev_check(P, launch_batch_in(B->nleaf, B->d_leafslot, B->d_leafhier, B->d_base,
                                          (const double* const*)B->d_ptrs, B->d_mass, st),
                       "batch gather")))
      return r;
    return run_solve(P, B->d_mass, T.lmax - 1, T.lmin_all, T.lmax, B->d_phi, B->d_acc, st);
  };
  if ((s = autotune_core(P, solve, st, out))) return s;
  if (hipStreamSynchronize(st) != hipSuccess) return fail(AFMM_E_DEVICE, "autotune sync");
  // kernel arguments and grids changed: capture the graph again
  return capture_batch(B);
}

// ---------------------------------------------------------------------------
// Adjoint pass.  Its topology (the source tiles of the transposed M2P / M2L and
// their tap splits) is built once; its per-call scratch -- target bars and mass
// bars on every level, source-copy / multipole bars on the multipole levels
// 2..lmax-1, local-expansion bars on the FMM levels 3..lmax-1, the transposed
// operators' B staging (tbT, lbarT) and the tap-split partial sets -- is laid
// out in one block: allocated by the plan on the first afmm_solve_adjoint, or
// taken from the library's static scratch array by afmm_solve_adjoint_noalloc.

static int device_cu_count() {
  int ncu = 256, dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  return ncu > 0 ? ncu : 256;
}

static afmm_status adjoint_topology(afmm_plan* P) {
  if (P->adj_topo) return AFMM_OK;
  const Topology& T = P->topo;
  afmm_status s;
  // source tiles: the level-ls cells read by some group of `grp` (refined ranks
  // at ls), 16 per tile in Morton order, one octant class per tile.  For every
  // tile, the taps (transposed order) whose group has a target child in some
  // column go to *livetaps (the kernel's own test, for the work estimate).
  // (Sorting the cells of a class by the side from which their groups lie
  // leaves more taps without a group in any column of a tile, but the tiles
  // lose the locality of their B rows, and the kernels ran slower.)
  using TapBits = std::array<uint64_t, 3>;
  auto src_tiles = [&](int target, const std::vector<int32_t>& grp, int32_t** dst, int* nt, uint8_t** live,
                       std::vector<TapBits>* livetaps) -> afmm_status {
    *nt = 0;
    livetaps->clear();
    if (grp.empty() || target < 3) return AFMM_OK;
    const int ls = target - 1;
    const HostLevel& LS = T.lv[ls];
    const HostLevel& LP = T.lv[ls - 1];
    std::vector<uint8_t> mark(LS.n(), 0);
    std::vector<uint8_t> flag(LS.nref(), 0);
    for (int32_t F : grp) {
      flag[F] = 1;
      const int32_t cF = LS.refcell[F];
      const int32_t G = cF >> 3, oF = cF & 7;
      for (int i = 0; i < kTapsPerClass; ++i) {
        const int code = P->tabs->taps[oF * kTapsPerClass + i];
        const int32_t Q = LP.nbr[(size_t)G * 27 + (code & 31)];
        if (Q < 0 || LP.rank[Q] < 0) continue;
        mark[8 * LP.rank[Q] + ((code >> 5) & 7)] = 1;
      }
    }
    std::vector<int32_t> cls[8], rec;
    for (int32_t c = 0; c < LS.n(); ++c)
      if (mark[c]) cls[c & 7].push_back(c);
    size_t chunks = 0;
    for (auto& c : cls) chunks = std::max(chunks, (c.size() + 15) / 16);
    for (size_t ch = 0; ch < chunks; ++ch)
      for (auto& c : cls) {
        if (ch * 16 >= c.size()) continue;
        rec.push_back(target);
        for (int j = 0; j < 16; ++j) rec.push_back(ch * 16 + j < c.size() ? c[ch * 16 + j] : -1);
        ++*nt;
      }
    livetaps->assign(*nt, TapBits{0, 0, 0});
    for (int t = 0; t < *nt; ++t) {
      const int32_t* col = &rec[(size_t)t * 17 + 1];
      const int os = col[0] & 7;
      for (int j = 0; j < kTapsPerClass; ++j) {
        const int code = P->tabs->tapsT[os * kTapsPerClass + j];
        for (int n = 0; n < 16; ++n) {
          if (col[n] < 0) continue;
          const int32_t Q = LP.nbr[(size_t)(col[n] >> 3) * 27 + (code & 31)];
          if (Q < 0 || LP.rank[Q] < 0) continue;
          const int32_t rF = LS.rank[8 * LP.rank[Q] + ((code >> 5) & 7)];
          if (rF >= 0 && flag[rF]) {
            (*livetaps)[t][j >> 6] |= 1ull << (j & 63);
            break;
          }
        }
      }
    }
    afmm_status s2 = upload(P, rec, dst, nullptr);
    return s2 ? s2 : upload(P, flag, live, nullptr);
  };
  // XCD ranges of equal estimated work: an item (tile, tap chunk) costs its
  // live taps plus a fixed setup worth kItemSetupTaps taps.
  auto xcd_ranges = [](const std::vector<TapBits>& bits, int ns) {
    constexpr double kItemSetupTaps = 3.0;
    XcdRanges xr;
    const int items = (int)bits.size() * ns;
    std::vector<double> cum(items + 1, 0.0);
    for (int i = 0; i < items; ++i) {
      const int t = i / ns, c = i - t * ns;
      const int lo = c * kTapsPerClass / ns, hi = (c + 1) * kTapsPerClass / ns;
      int live = 0;
      for (int j = lo; j < hi; ++j) live += (int)((bits[t][j >> 6] >> (j & 63)) & 1);
      cum[i + 1] = cum[i] + live + kItemSetupTaps;
    }
    for (int x = 0; x <= 8; ++x)
      xr.start[x] = x == 8 ? items
                           : (int32_t)(std::lower_bound(cum.begin(), cum.end(), cum[items] * x / 8.0) - cum.begin());
    for (int x = 1; x <= 8; ++x) xr.start[x] = std::max(xr.start[x], xr.start[x - 1]);
    return xr;
  };
  std::vector<TapBits> bits_p[kMaxLevel], bits_l[kMaxLevel];
  for (int l = 3; l <= T.lmax; ++l)
    if ((s = src_tiles(l, T.leafgrp[l], &P->d_adjp[l], &P->n_adjp[l], &P->d_adjp_live[l], &bits_p[l]))) return s;
  for (int f = 3; f <= T.lmax - 1; ++f)
    if ((s = src_tiles(f, T.m2lgrp[f], &P->d_adjl[f], &P->n_adjl[f], &P->d_adjl_live[f], &bits_l[f]))) return s;
  // tap splits of the transposed translations: about 24 work items per CU, so
  // that the items left after the first wave of workgroups even out the CUs
  // (tiles differ in their number of live taps)
  const int ncu = device_cu_count();
  auto split_of = [&](int nt) { return nt > 0 ? std::max(1, std::min(16, (24 * ncu + nt - 1) / nt)) : 1; };
  P->adj_part_elems = 0;
  for (int l = 0; l < kMaxLevel; ++l) {
    P->s_adjp[l] = split_of(P->n_adjp[l]);
    P->s_adjl[l] = split_of(P->n_adjl[l]);
    P->xr_adjp[l] = xcd_ranges(bits_p[l], P->s_adjp[l]);
    P->xr_adjl[l] = xcd_ranges(bits_l[l], P->s_adjl[l]);
    if (P->s_adjp[l] > 1) P->adj_part_elems = std::max(P->adj_part_elems, (size_t)P->s_adjp[l] * P->n_adjp[l] * 16 * P->K);
    if (P->s_adjl[l] > 1) P->adj_part_elems = std::max(P->adj_part_elems, (size_t)P->s_adjl[l] * P->n_adjl[l] * 16 * P->K);
  }
  P->adj_topo = true;
  return AFMM_OK;
}

// Lays the adjoint scratch out from `base` (256-byte aligned pieces) into the
// bar pointers of lw[] (a copy of the plan's levels) and *part; returns the
// bytes used.  With base == nullptr only the size is computed.
static size_t adjoint_layout(const afmm_plan* P, char* base, LevelDev* lw, double** part) {
  const Topology& T = P->topo;
  const int K = P->K;
  const bool mixed = P->opt.precision == AFMM_FP32_MIXED;
  const int f64 = mixed ? P->opt.fp64_levels : 1 << 20;
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* q = base ? (void*)(base + off) : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return q;
  };
  for (int l = 0; l <= T.lmax; ++l) {
    LevelDev& D = lw[l];
    D.tbar = (double*)take((size_t)std::max(D.n, 1) * 4 * sizeof(double));
    D.mbar = (double*)take((size_t)std::max(D.n, 1) * sizeof(double));
    D.sbar = (l >= 2 && l <= T.lmax - 1 && D.nref > 0) ? (double*)take((size_t)D.nref * K * sizeof(double)) : nullptr;
    D.lbar = (l >= P->l_first && l <= T.lmax - 1 && D.nref > 0) ? (double*)take((size_t)D.nref * K * sizeof(double))
                                                                  : nullptr;
    D.tbT = nullptr;
    D.lbarT = nullptr;
  }
  for (int l = 3; l <= T.lmax; ++l)
    if (P->n_adjp[l] > 0) {
      const size_t es = (mixed && (l - 1) > f64) ? sizeof(float) : sizeof(double);
      lw[l - 1].tbT = take((size_t)T.lv[l - 1].nref() * 32 * es);
    }
  for (int f = 3; f <= T.lmax - 1; ++f)
    if (P->n_adjl[f] > 0) {
      const bool f32 = mixed && f > f64;
      lw[f].lbarT = take((size_t)T.lv[f].nref() *
                         (f32 ? src_row(P->opt.p, 4) * sizeof(float) : src_row(P->opt.p, 8) * sizeof(double)));
    }
  *part = P->adj_part_elems ? (double*)take(P->adj_part_elems * sizeof(double)) : nullptr;
  return off;
}

// The plan-owned scratch of afmm_solve_adjoint (allocated on its first call).
static afmm_status adjoint_workspace(afmm_plan* P) {
  if (P->adj_ready) return AFMM_OK;
  afmm_status s;
  if ((s = adjoint_topology(P))) return s;
  if (hipDeviceSynchronize() != hipSuccess) return fail(AFMM_E_DEVICE, "adjoint topology upload");
  double* part = nullptr;
  const size_t bytes = adjoint_layout(P, nullptr, P->lv, &part);
  void* q = nullptr;
  if ((s = dev_alloc(P, &q, bytes))) return s;
  adjoint_layout(P, (char*)q, P->lv, &part);
  P->adj_part = part;
  P->adj_ready = true;
  return AFMM_OK;
}

// The adjoint of the last solve (Alg. 1-4 transposed) with the bars and
// partial sets of lw[] / part.
static afmm_status run_adjoint(afmm_plan* P, int32_t level, const double* d_phi_bar, const double* d_acc_bar,
                               double* d_mass_bar, hipStream_t st, const LevelDev* lw, double* part) {
  const Topology& T = P->topo;
  const int p = P->opt.p, K = P->K;
  const int lmin = T.levelmin[0], lmax = T.lmax;
  const int lo = level == AFMM_ALL_LEVELS ? lmin : level, hi = level == AFMM_ALL_LEVELS ? lmax : level;
  const int fmax = hi - 1;
  afmm_status s;
  const WorkCounts& W = P->work;
  // 1. unit-form bars of the targets, zeroed accumulators
  hipEvent_t ev = prof_begin(P, st);
  for (int l = 0; l <= lmax; ++l) {
    const double h = P->opt.boxlen / (double)(1LL << l);
    const bool tgt = l >= lo && l <= hi;
    if ((s = dev_check(P, launch_adj_init(lw[l], tgt, d_phi_bar, d_acc_bar, P->opt.G / h, P->opt.G / (h * h), st),
                       "adjoint init")))
      return s;
    if ((s = dev_check(P, launch_adj_zero(lw[l].sbar, lw[l].sbar ? (size_t)lw[l].nref * K : 0, st),
                       "adjoint zero")) ||
        (s = dev_check(P, launch_adj_zero(lw[l].lbar, lw[l].lbar ? (size_t)lw[l].nref * K : 0, st),
                       "adjoint zero")))
      return s;
  }
  prof_end(P, ev, st, kAdjTree, -1);
  // 2. leaf fields: P2P^T into the mass bars of every level next to a target
  //    level, near M2P^T and L2P^T of the target levels
  const LevelDev empty;
  ev = prof_begin(P, st);
  for (int l = lo; l <= hi; ++l) {
    P->pending_flops += W.leaf_flops[l];
    P->pending_bytes += W.leaf_bytes[l];
  }
  for (int l = std::max(1, lo - 1); l <= std::min(lmax, hi + 1); ++l) {
    const LevelDev& lvp = l + 1 <= lmax ? lw[l + 1] : empty;
    const bool tgt = l >= lo && l <= hi;
    // P2P^T over the groups with a leaf child; near M2P^T over the groups with a
    // refined child (the M2L group list from level 3 on, every refined cell below)
    const int nlg = (int)T.leafgrp[l].size();
    const int nrg = l >= 3 ? (int)T.m2lgrp[l].size() : lw[l - 1].nref;
    if ((s = dev_check(P,
                       launch_adj_near(p, P->d_leafgrp[l], nlg, P->d_adjvgrp[l], (int)T.adjvgrp[l].size(),
                                       l >= 3 ? P->d_m2lgrp[l] : nullptr, nrg, lw[l - 1], lw[l], lvp, tgt,
                                       P->t64, P->cm, st),
                       "adjoint near")))
      return s;
    if (tgt && l - 1 >= P->l_first && lw[l - 1].lbar &&
        (s = dev_check(P, launch_adj_l2p(p, P->d_leafgrp[l], nlg, lw[l - 1], lw[l], P->t64, P->cm, st),
                       "adjoint l2p")))
      return s;
  }
  prof_end(P, ev, st, kAdjNear, -1);
  // 3. intermediate field: M2P^T into the level l-1 sources
  ev = prof_begin(P, st);
  const bool mixed = P->opt.precision == AFMM_FP32_MIXED;
  const int f64 = mixed ? P->opt.fp64_levels : 1 << 20;
  for (int l = std::max(3, lo); l <= hi; ++l) {
    if ((s = dev_check(P,
                       launch_adj_m2p_mfma(p, mixed && (l - 1) > f64, P->d_adjp[l], P->n_adjp[l], P->s_adjp[l],
                                           P->xr_adjp[l], P->d_adjp_live[l], part,
                                           P->cm.tapsT, P->cm.adj_m2p_off, lw[l - 2], lw[l - 1], lw[l], P->t32, P->t64,
                                           st),
                       "adjoint m2p")))
      return s;
    P->pending_flops += W.m2p_flops[l];
    P->pending_bytes += W.m2p_bytes[l];
  }
  prof_end(P, ev, st, kAdjM2P, -1);
  // 4. L2L^T, finest FMM level first (into the first level with local expansions)
  ev = prof_begin(P, st);
  for (int f = fmax; f >= P->l_first + 1; --f)
    if ((s = dev_check(P,
                       launch_adj_l2l(p, P->d_m2lgrp[f], (int)T.m2lgrp[f].size(), lw[f - 1], lw[f], P->t64, P->cm,
                                      st),
                       "adjoint l2l")))
      return s;
  prof_end(P, ev, st, kAdjTree, -1);
  // 5. M2L^T into the level f-1 sources
  ev = prof_begin(P, st);
  for (int f = 3; f <= fmax; ++f) {
    if ((s = dev_check(P,
                       launch_adj_m2l_mfma(p, mixed && f > f64, P->d_adjl[f], P->n_adjl[f], P->s_adjl[f],
                                           P->xr_adjl[f], P->d_adjl_live[f], part,
                                           P->cm.tapsT, P->cm.adj_m2l_off, lw[f - 2], lw[f - 1], lw[f], P->t32, P->t64,
                                           st),
                       "adjoint m2l")))
      return s;
    P->pending_flops += W.m2l_flops[f];
    P->pending_bytes += W.m2l_bytes[f];
  }
  prof_end(P, ev, st, kAdjM2L, -1);
  ev = prof_begin(P, st);
  // 6. source-copy bars -> multipole bars, M2M^T coarse to fine; with periodic
  //    boxes the transposed level-2 far operator joins the level-2 multipole bars
  //    before they pass down
  for (int f = 2; f <= lmax - 1; ++f) {
    if ((s = dev_check(P,
                       launch_adj_down(p, P->d_upmix[f - 1], (int)T.upmix[f - 1].size(), lw[f - 1], lw[f], f >= 3,
                                       P->cm, st),
                       "adjoint down")))
      return s;
    if (f == 2 && T.periodic && fmax >= 2 &&
        (s = dev_check(P, launch_adj_periodic_far(p, lw[2], P->d_pfar, P->d_pfar_cf, P->cm, st),
                       "adjoint periodic far")))
      return s;
  }
  // 7. mass bars to the caller's slots (levels whose masses came from the last call)
  for (int l = lmin; l <= lmax; ++l) {
    const bool has_parent = l - 1 >= 2 && l - 1 <= lmax - 1;
    const bool fresh = l >= P->last_fresh;
    if ((s = dev_check(P, launch_adj_out(p, lw[l - 1], lw[l], has_parent, fresh, P->cself, P->cm, d_mass_bar, st),
                       "adjoint out")))
      return s;
  }
  prof_end(P, ev, st, kAdjTree, -1);
  return AFMM_OK;
}

static afmm_status adjoint_args(afmm_plan* P, int32_t level, const double* d_phi_bar, const double* d_acc_bar,
                                double* d_mass_bar) {
  if (!P || !d_phi_bar || !d_acc_bar || !d_mass_bar) return fail(AFMM_E_INVALID_ARG, "null argument");
  if (P->dead) return fail(AFMM_E_DEVICE, "plan is unusable after an earlier device error");
  if (P->topo.levelmin.size() != 1) return fail(AFMM_E_INVALID_ARG, "batched plan: no adjoint");
  if (!P->solved) return fail(AFMM_E_ATS_ORDER, "adjoint before any solve");
  if (level != P->last_level) return fail(AFMM_E_INVALID_ARG, "adjoint level differs from the last solve's level");
  return AFMM_OK;
}

static afmm_status afmm_solve_adjoint_impl(afmm_plan* P, int32_t level, const double* d_phi_bar,
                                          const double* d_acc_bar, double* d_mass_bar, void* hip_stream) {
  afmm_status s;
  if ((s = adjoint_args(P, level, d_phi_bar, d_acc_bar, d_mass_bar))) return s;
  if ((s = adjoint_workspace(P))) return s;
  return run_adjoint(P, level, d_phi_bar, d_acc_bar, d_mass_bar, (hipStream_t)hip_stream, P->lv, P->adj_part);
}

// ---------------------------------------------------------------------------
// Allocation-free adjoint.  Its scratch lives in `scratch`, a file-scope
// device array of kScratchBytes: every GPU the library runs on holds one copy
// until the process ends.  Host code never uses the array's name as an address
// (on the host it is only a stand-in for the symbol): the device address of
// each GPU's copy is looked up once per device with hipGetSymbolAddress and
// kept in g_scratch_ptr.  Every call on one GPU shares its copy, so calls that
// overlap on one GPU (other streams, other threads) race; calls on one stream
// are ordered.  Every byte a call reads is written earlier in the same call
// (bars are cleared by fill kernels, the B staging and the partial sets are
// written in full), so no call depends on what the previous one left.
namespace {
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
}  // namespace
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static void* g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

static afmm_status scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(AFMM_E_DEVICE, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices) return fail(AFMM_E_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return fail(AFMM_E_DEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return AFMM_OK;
}

// Whether the allocation-free adjoint can serve this plan, from an upper bound
// of its scratch that needs no topology: every level with B staging, and tap
// -split partial sets for tile counts of at most ceil(cells / 16) + 8.
static bool adjoint_noalloc_may_fit(const afmm_plan* P) {
  const Topology& T = P->topo;
  const int K = P->K;
  size_t b = 0;
  auto add = [&](size_t bytes) { b += (bytes + 255) & ~(size_t)255; };
  const int ncu = device_cu_count();
  size_t part = 0;
  for (int l = 0; l <= T.lmax; ++l) {
    const size_t n = (size_t)std::max(T.lv[l].n(), 1), nref = (size_t)T.lv[l].nref();
    add(n * 32);
    add(n * 8);
    add(nref * K * 8);
    add(nref * K * 8);
    add(nref * 32 * 8);
    add(nref * (size_t)src_row(P->opt.p, 8) * 8);
    const size_t nt = (size_t)(T.lv[l].n() + 15) / 16 + 8;
    const size_t sp = (size_t)std::max(1, std::min(16, (int)((12 * (size_t)ncu + nt - 1) / nt)));
    part = std::max(part, sp * nt * 16 * K);
  }
  add(part * 8);
  return b <= kScratchBytes;
}

static afmm_status afmm_solve_adjoint_noalloc_impl(afmm_plan* P, int32_t level, const double* d_phi_bar,
                                                  const double* d_acc_bar, double* d_mass_bar, void* hip_stream) {
  afmm_status s;
  if ((s = adjoint_args(P, level, d_phi_bar, d_acc_bar, d_mass_bar))) return s;
  if (!P->adj_topo)
    return fail(AFMM_E_OUT_OF_MEMORY,
                "the plan's adjoint scratch exceeds the static maximum of afmm_solve_adjoint_noalloc (its topology "
                "was not prepared at plan creation)");
  LevelDev lw[kMaxLevel + 1];
  std::memcpy((void*)lw, (const void*)P->lv, sizeof lw);
  double* part = nullptr;
  const size_t need = adjoint_layout(P, nullptr, lw, &part);
  if (need > kScratchBytes) {
    char b[200];
    snprintf(b, sizeof b, "adjoint scratch of %zu bytes exceeds the static maximum of %zu bytes", need, kScratchBytes);
    return fail(AFMM_E_OUT_OF_MEMORY, b);
  }
  void* base = nullptr;
  if ((s = scratch_address(&base))) return s;
  adjoint_layout(P, (char*)base, lw, &part);
  return run_adjoint(P, level, d_phi_bar, d_acc_bar, d_mass_bar, (hipStream_t)hip_stream, lw, part);
}

// Append topology S (one hierarchy) to the forest T, offsetting cells, refined
// ranks and slots.  Level l of S holds 8 x (refined cells of level l-1) cells
// like T, so the children of a shifted refined rank stay at 8r..8r+7.
static void merge_topology(Topology& T, const Topology& S, int64_t slot_base) {
  for (int l = 0; l <= S.lmax; ++l) {
    HostLevel& D = T.lv[l];
    const HostLevel& E = S.lv[l];
    const int32_t base = D.n(), rbase = D.nref();
    for (int32_t c = 0; c < E.n(); ++c) {
      D.rank.push_back(E.rank[c] >= 0 ? E.rank[c] + rbase : -1);
      D.slot.push_back(E.slot[c] >= 0 ? (int32_t)(E.slot[c] + slot_base) : -1);
    }
    for (int32_t r = 0; r < E.nref(); ++r) D.refcell.push_back(E.refcell[r] + base);
    for (int32_t v : E.nbr) D.nbr.push_back(v >= 0 ? v + base : v);
  }
  T.lmax = std::max(T.lmax, S.lmax);
  for (size_t i = 0; i < S.levelmin.size(); ++i) {
    T.lmin_all = std::min(T.lmin_all, S.levelmin[i]);
    T.levelmin.push_back(S.levelmin[i]);
    T.levelmax.push_back(S.levelmax[i]);
    T.slot_base.push_back(slot_base + S.slot_base[i]);
    T.slot_count.push_back(S.slot_count[i]);
    T.level_off.push_back(S.level_off[i]);
  }
  T.nslots = slot_base + S.nslots;
}

// Refresh the device table of caller pointers (stream-ordered, no host sync
// unless the previous refresh is still pending).
static afmm_status batch_pointer_table(afmm_batch* B, const double* const* d_mass, double* const* d_phi,
                                       double* const* d_acc, hipStream_t st) {
  const int32_t n = B->n;
  for (int32_t i = 0; i < n; ++i)
    if (!d_mass[i] || !d_phi[i] || !d_acc[i]) return fail(AFMM_E_INVALID_ARG, "null array in batch");
  if (hipEventSynchronize(B->ev_stage) != hipSuccess) return dev_check(B->plan, hipGetLastError(), "table event");
  for (int32_t i = 0; i < n; ++i) {
    B->h_stage[i] = (void*)d_mass[i];
    B->h_stage[n + i] = (void*)d_phi[i];
    B->h_stage[2 * n + i] = (void*)d_acc[i];
  }
  afmm_status s;
  if ((s = dev_check(B->plan, hipMemcpyAsync(B->d_ptrs, B->h_stage, (size_t)3 * n * sizeof(void*),
                                             hipMemcpyHostToDevice, st),
                     "batch pointer table")))
    return s;
  return dev_check(B->plan, hipEventRecord(B->ev_stage, st), "table event");
}

static void free_batch(afmm_batch* B) {
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  if (B->cap) (void)hipStreamDestroy(B->cap);
  if (B->ev_stage) {
    (void)hipEventSynchronize(B->ev_stage);
    (void)hipEventDestroy(B->ev_stage);
  }
  if (B->h_stage) (void)hipHostFree(B->h_stage);
  B->ev_stage = nullptr;
  B->h_stage = nullptr;
  if (B->plan) {
    free_plan(B->plan);
    delete B->plan;
  }
  B->exec = nullptr;
  B->graph = nullptr;
  B->cap = nullptr;
  B->plan = nullptr;
}

// Capture gather -> solve -> scatter of a batch into its graph (replacing an
// earlier one).
static afmm_status capture_batch(afmm_batch* B) {
  afmm_plan* P = B->plan;
  const Topology& T = P->topo;
  const int n = B->n;
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->exec = nullptr;
  B->graph = nullptr;
  const bool prof = P->profiling;
  P->profiling = false;
  hipStream_t cs = B->cap;
  afmm_status s = AFMM_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    s = fail(AFMM_E_DEVICE, "graph capture could not start");
  } else {
    afmm_status sr = dev_check(P, launch_batch_in(B->nleaf, B->d_leafslot, B->d_leafhier, B->d_base,
                                                  (const double* const*)B->d_ptrs, B->d_mass, cs),
                               "batch gather");
    if (!sr) sr = run_solve(P, B->d_mass, T.lmax - 1, T.lmin_all, T.lmax, B->d_phi, B->d_acc, cs);
    if (!sr)
      sr = dev_check(P, launch_batch_out(B->nleaf, B->d_leafslot, B->d_leafhier, B->d_base, B->d_phi, B->d_acc,
                                         (double* const*)(B->d_ptrs + n), (double* const*)(B->d_ptrs + 2 * n), cs),
                     "batch scatter");
    const hipError_t ee = hipStreamEndCapture(cs, &B->graph);
    if (sr) s = sr;
    else if (ee != hipSuccess || !B->graph) s = fail(AFMM_E_DEVICE, "graph capture failed");
    else if (hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0) != hipSuccess)
      s = fail(AFMM_E_DEVICE, "graph instantiation failed");
  }
  P->profiling = prof;
  return s;
}

static afmm_status afmm_batch_create_impl(afmm_plan* const* plans, int32_t n, void* hip_stream, afmm_batch** out) {
  if (!plans || !out || n < 1) return fail(AFMM_E_INVALID_ARG, "null argument or n < 1");
  *out = nullptr;
  hipStream_t st = (hipStream_t)hip_stream;
  const afmm_options& o0 = plans[0] ? plans[0]->opt : afmm_options{};
  for (int32_t i = 0; i < n; ++i) {
    const afmm_plan* Q = plans[i];
    if (!Q) return fail(AFMM_E_INVALID_ARG, "null plan in batch");
    if (Q->dead) return fail(AFMM_E_DEVICE, "a plan of the batch is unusable after a device error");
    if (Q->topo.levelmin.size() != 1) return fail(AFMM_E_INVALID_ARG, "a batch takes single-hierarchy plans");
    const afmm_options& o = Q->opt;
    const uint32_t kModel = AFMM_PAPER_QUAD_CAP | AFMM_SELF_POTENTIAL | AFMM_PERIODIC;
    if (o.p != o0.p || o.precision != o0.precision || o.G != o0.G || o.boxlen != o0.boxlen ||
        o.fp64_levels != o0.fp64_levels || o.tap_split != o0.tap_split || ((o.flags ^ o0.flags) & kModel))
      return fail(AFMM_E_INVALID_ARG,
                  "plans of a batch must share p, precision, G, boxlen, fp64_levels, tap_split and the "
                  "quadrupole-cap / self-potential / periodic flags");
  }
  afmm_batch* B = new afmm_batch();
  try {
    B->n = n;
    B->plan = new afmm_plan();
    afmm_plan* P = B->plan;
    P->opt = o0;
    P->opt.flags = o0.flags & (AFMM_PAPER_QUAD_CAP | AFMM_SELF_POTENTIAL | AFMM_PERIODIC);
    P->K = nmi(o0.p);
    P->topo.periodic = (o0.flags & AFMM_PERIODIC) != 0;
    B->base.assign(n + 1, 0);
    for (int32_t i = 0; i < n; ++i) {
      merge_topology(P->topo, plans[i]->topo, B->base[i]);
      B->base[i + 1] = B->base[i] + plans[i]->topo.nslots;
    }
    afmm_status s = B->base[n] >= ((int64_t)1 << 31) ? fail(AFMM_E_INVALID_ARG, "batch has more than 2^31 cells")
                                                      : plan_finish(P, st);
    // leaf slots of the forest and their hierarchy
    std::vector<int32_t> lslot, lhier;
    if (!s) {
      const Topology& T = P->topo;
      for (int l = 0; l <= T.lmax; ++l)
        for (int32_t c = 0; c < T.lv[l].n(); ++c) {
          const int32_t sl = T.lv[l].slot[c];
          if (T.lv[l].rank[c] >= 0 || sl < 0) continue;
          lslot.push_back(sl);
          lhier.push_back((int32_t)(std::upper_bound(B->base.begin(), B->base.end(), (int64_t)sl) - B->base.begin() - 1));
        }
      B->nleaf = (int64_t)lslot.size();
      void* q = nullptr;
      const size_t ns = (size_t)std::max<int64_t>(P->topo.nslots, 1);
      if (!s) s = dev_alloc(P, &q, ns * sizeof(double)), B->d_mass = (double*)q;
      if (!s) s = dev_alloc(P, &q, ns * sizeof(double)), B->d_phi = (double*)q;
      if (!s) s = dev_alloc(P, &q, ns * 3 * sizeof(double)), B->d_acc = (double*)q;
      if (!s) s = dev_alloc(P, &q, (size_t)3 * n * sizeof(void*)), B->d_ptrs = (void**)q;
      if (!s) s = upload(P, lslot, &B->d_leafslot, st);
      if (!s) s = upload(P, lhier, &B->d_leafhier, st);
      if (!s) s = upload(P, B->base, &B->d_base, st);
      if (!s && (hipHostMalloc((void**)&B->h_stage, (size_t)3 * n * sizeof(void*), hipHostMallocDefault) != hipSuccess ||
                 hipEventCreateWithFlags(&B->ev_stage, hipEventDisableTiming) != hipSuccess ||
                 hipEventRecord(B->ev_stage, st) != hipSuccess))
        s = fail(AFMM_E_DEVICE, "batch pointer staging");
    }
    // capture: gather -> solve -> scatter, replayed by afmm_batch_solve
    if (!s) {
      if (hipStreamSynchronize(st) != hipSuccess ||
          hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking) != hipSuccess)
        s = fail(AFMM_E_DEVICE, "batch stream creation failed");
    }
    if (!s) s = capture_batch(B);
    if (s) {
      free_batch(B);
      delete B;
      return s;
    }
  } catch (...) {
    free_batch(B);
    delete B;
    throw;
  }
  *out = B;
  return AFMM_OK;
}

static afmm_status afmm_batch_solve_impl(afmm_batch* B, const double* const* d_mass, double* const* d_phi,
                                        double* const* d_acc, void* hip_stream) {
  if (!B || !d_mass || !d_phi || !d_acc) return fail(AFMM_E_INVALID_ARG, "null argument");
  if (B->plan->dead) return fail(AFMM_E_DEVICE, "batch is unusable after an earlier device error");
  const int32_t n = B->n;
  hipStream_t st = (hipStream_t)hip_stream;
  afmm_status s;
  if ((s = batch_pointer_table(B, d_mass, d_phi, d_acc, st))) return s;
  afmm_plan* P = B->plan;
  if (!P->profiling) return dev_check(P, hipGraphLaunch(B->exec, st), "batch graph launch");
  // profiled solves run the same launches eagerly, each bracketed by events
  const Topology& T = P->topo;
  if ((s = dev_check(P, launch_batch_in(B->nleaf, B->d_leafslot, B->d_leafhier, B->d_base,
                                        (const double* const*)B->d_ptrs, B->d_mass, st),
                     "batch gather")) ||
      (s = run_solve(P, B->d_mass, T.lmax - 1, T.lmin_all, T.lmax, B->d_phi, B->d_acc, st)))
    return s;
  return dev_check(P, launch_batch_out(B->nleaf, B->d_leafslot, B->d_leafhier, B->d_base, B->d_phi, B->d_acc,
                                       (double* const*)(B->d_ptrs + n), (double* const*)(B->d_ptrs + 2 * n), st),
                   "batch scatter");
}

extern "C" afmm_status afmm_batch_set_profiling(afmm_batch* B, int32_t enable) {
  if (!B) return fail(AFMM_E_INVALID_ARG, "null batch");
  return afmm_plan_set_profiling(B->plan, enable);
}

static afmm_status afmm_batch_get_profile_impl(afmm_batch* B, afmm_stage_time* out, int32_t cap, int32_t* n_out) {
  if (!B) return fail(AFMM_E_INVALID_ARG, "null batch");
  return afmm_plan_get_profile(B->plan, out, cap, n_out);
}

extern "C" afmm_status afmm_batch_get_info(const afmm_batch* B, afmm_plan_info* out) {
  if (!B || !out) return fail(AFMM_E_INVALID_ARG, "null argument");
  if (afmm_status s = ensure_info(B->plan)) return s;
  *out = B->plan->info;
  out->device_bytes = B->plan->bytes;
  return AFMM_OK;
}

extern "C" afmm_status afmm_batch_destroy(afmm_batch* B) {
  if (!B) return AFMM_OK;
  if (B->plan && B->plan->side) (void)hipStreamSynchronize(B->plan->side);
  if (B->cap) (void)hipStreamSynchronize(B->cap);
  free_batch(B);
  delete B;
  return AFMM_OK;
}

// ---------------------------------------------------------------------------
// C ABI entry points that allocate: exceptions become status codes.

extern "C" afmm_status afmm_plan_create(const afmm_hierarchy* h, const afmm_options* opt, void* hip_stream,
                                        afmm_plan** out) {
  return guarded([&] { return afmm_plan_create_impl(h, opt, hip_stream, out); });
}

extern "C" afmm_status afmm_plan_replan(const afmm_plan* old, const afmm_hierarchy* h, int32_t level, void* hip_stream,
                                        afmm_plan** out) {
  return guarded([&] { return afmm_plan_replan_impl(old, h, level, hip_stream, out); });
}

extern "C" afmm_status afmm_solve(afmm_plan* P, int32_t level, int32_t icount, const double* d_mass, double* d_phi,
                                  double* d_acc, void* hip_stream) {
  return guarded([&] { return afmm_solve_impl(P, level, icount, d_mass, d_phi, d_acc, hip_stream); });
}

extern "C" afmm_status afmm_solve_drift(afmm_plan* P, int32_t level, int32_t icount, double time,
                                        const double* d_mass, const double* d_mass_rate, double* d_phi, double* d_acc,
                                        void* hip_stream) {
  if (!d_mass_rate) return fail(AFMM_E_INVALID_ARG, "null mass rate");
  return guarded(
      [&] { return afmm_solve_impl(P, level, icount, d_mass, d_phi, d_acc, hip_stream, time, d_mass_rate); });
}

extern "C" afmm_status afmm_plan_get_profile(afmm_plan* P, afmm_stage_time* out, int32_t cap, int32_t* n_out) {
  return guarded([&] { return afmm_plan_get_profile_impl(P, out, cap, n_out); });
}

extern "C" afmm_status afmm_plan_autotune(afmm_plan* P, const double* d_mass, double* d_phi, double* d_acc,
                                          void* hip_stream, afmm_tune_result* out) {
  return guarded([&] { return afmm_plan_autotune_impl(P, d_mass, d_phi, d_acc, hip_stream, out); });
}

extern "C" afmm_status afmm_batch_autotune(afmm_batch* B, const double* const* d_mass, double* const* d_phi,
                                           double* const* d_acc, void* hip_stream, afmm_tune_result* out) {
  return guarded([&] { return afmm_batch_autotune_impl(B, d_mass, d_phi, d_acc, hip_stream, out); });
}

extern "C" afmm_status afmm_solve_adjoint(afmm_plan* P, int32_t level, const double* d_phi_bar,
                                          const double* d_acc_bar, double* d_mass_bar, void* hip_stream) {
  return guarded([&] { return afmm_solve_adjoint_impl(P, level, d_phi_bar, d_acc_bar, d_mass_bar, hip_stream); });
}

extern "C" afmm_status afmm_solve_adjoint_noalloc(afmm_plan* P, int32_t level, const double* d_phi_bar,
                                                  const double* d_acc_bar, double* d_mass_bar, void* hip_stream) {
  return guarded(
      [&] { return afmm_solve_adjoint_noalloc_impl(P, level, d_phi_bar, d_acc_bar, d_mass_bar, hip_stream); });
}

extern "C" afmm_status afmm_batch_create(afmm_plan* const* plans, int32_t n, void* hip_stream, afmm_batch** out) {
  return guarded([&] { return afmm_batch_create_impl(plans, n, hip_stream, out); });
}

extern "C" afmm_status afmm_batch_solve(afmm_batch* B, const double* const* d_mass, double* const* d_phi,
                                        double* const* d_acc, void* hip_stream) {
  return guarded([&] { return afmm_batch_solve_impl(B, d_mass, d_phi, d_acc, hip_stream); });
}

extern "C" afmm_status afmm_batch_get_profile(afmm_batch* B, afmm_stage_time* out, int32_t cap, int32_t* n_out) {
  return guarded([&] { return afmm_batch_get_profile_impl(B, out, cap, n_out); });
}

extern "C" afmm_status afmm_hierarchy_check(const afmm_hierarchy* h, const afmm_options* opt, afmm_plan_info* out) {
  return guarded([&] { return afmm_hierarchy_check_impl(h, opt, out); });
}

// ---------------------------------------------------------------------------
// plan services of the particle-mesh calls (afmm_pm.hip)

namespace afmm {

afmm_status pm_fail(afmm_status s, const char* msg) { return fail(s, msg); }

double plan_boxlen(const afmm_plan* P) { return P->opt.boxlen; }

afmm_status plan_pm_flag(afmm_plan* P, int** d_flag, int** h_flag) {
  if (P->dead) return fail(AFMM_E_DEVICE, "plan is unusable after an earlier device error");
  *d_flag = P->d_flag;
  *h_flag = P->h_flag;
  return AFMM_OK;
}

// Morton keys of the cells of level `level` in the plan's order: the children
// of refined rank r are cells 8r..8r+7 in octant order, so key = (father's
// key << 3) | octant, ascending level by level.  Built on the host and uploaded
// the first time a level is asked for (8 bytes per cell of that level).
afmm_status plan_level_keys(afmm_plan* P, int level, const uint64_t** keys, const LevelDev** lv) {
  if (P->dead) return fail(AFMM_E_DEVICE, "plan is unusable after an earlier device error");
  const Topology& T = P->topo;
  if (T.levelmin.size() != 1) return fail(AFMM_E_INVALID_ARG, "batched plan: no particle-mesh calls");
  if (level < T.levelmin[0] || level > T.lmax) return fail(AFMM_E_INVALID_ARG, "level outside [levelmin, levelmax]");
  if (!P->d_keys[level]) {
    std::vector<uint64_t> prev{0}, cur;
    for (int l = 1; l <= level; ++l) {
      const HostLevel& U = T.lv[l - 1];
      cur.assign((size_t)T.lv[l].n(), 0);
      for (int32_t r = 0; r < U.nref(); ++r)
        for (int o = 0; o < 8; ++o) cur[(size_t)8 * r + o] = (prev[U.refcell[r]] << 3) | (uint64_t)o;
      prev.swap(cur);
    }
    uint64_t* d = nullptr;
    afmm_status s = upload(P, prev, &d, nullptr);
    if (s) return s;
    P->d_keys[level] = d;
  }
  *keys = P->d_keys[level];
  *lv = &P->lv[level];
  return AFMM_OK;
}

}  // namespace afmm
