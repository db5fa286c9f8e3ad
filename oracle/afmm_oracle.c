/*
 * afmm_oracle.c -- plain FP64 CPU reference of the adaptive FMM Poisson solver
 * of Lee & Teyssier, "A Scalable FMM Poisson Solver for the RAMSES code: II.
 * Adaptive Mesh Refinement and Adaptive Time Stepping".
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP solver.
 *
 * What it computes (the paper's notation):
 *   - one FMM tree T_j per AMR level j (Sec. 3.1); T_j accumulates only the
 *     leaves of level j, its FMM grid T_{j;f} has levels 1 <= f <= j-1, and
 *     M_{j;j} are the level-j leaf masses;
 *   - multipoles by their definition (Sec. 2, Eq. eqn:multipole): raw moments
 *     M_a = sum m (x - c)^a about the geometric centre c of each FMM cell
 *     (the M2M chain of Eq. eq:M2M_general is provided separately, for a pin);
 *   - the merged tree  ~T_{l+1} = sum_{j>l} T_j  (Sec. 3.1/3.3, Alg. 1);
 *   - Alg. 3 MultipoleToLocal: L_{l;f} = ShiftLocal(L_{l;f-1})
 *       + sum_{j=max(lmin,f-1)}^{l} K M_{j;f-1} + K ~M_{l+1;f-1},
 *     applied tree by tree over the interaction list (Sec. 2: the 6^3 block
 *     around the father's oct minus the 3^3 cells touching the father);
 *   - Alg. 4 PotentialEvaluation, read through the field anatomy of Sec. 3.2
 *     (figure fig:field): far = L2P of L_{l;l-1}; intermediate = P2P from
 *     level-(l-1) leaves + M2P from T_{l;l-1} + M2P from ~T_{l+1;l-1}; near =
 *     P2P from level-(l-1) and level-l leaves + M2P from ~T_{l+1;l} for refined
 *     level-l cells not touching the target; nearest = P2P from the 8 children
 *     of refined level-l cells touching the target;
 *   - Alg. 1 / Alg. 2 life cycle for adaptive time stepping: trees j >= l are
 *     rebuilt iff l == levelmin or icount > 1; stale trees keep both their
 *     multipoles and their leaf masses.
 *
 * Readings where the paper is silent (listed with the others in the design
 * notes): g(R) = -G/|R|, R = target - source, a = -grad(phi); multipoles and
 * local expansions truncated at total order p (|a|+|b| <= p in Eq. eq:M2L),
 * forces therefore use multipoles up to order p-1; the level-f targets of
 * M2L take sources one level coarser (the Delta-l = 1 footnote of Sec. 2);
 * L = 0 on FMM level 1; isolated box, lists clipped to [0, boxlen)^3; no
 * self-interaction; only leaves are targets.
 *
 * Periodic boundaries (an extension: Sec. 5 names periodic domains as future
 * work; readings in the design notes).  The box is a torus and the potential
 * that of the masses with a uniform neutralising background, zero on average
 * (the Ewald sum, oracle_direct_periodic).  The FMM then wraps every cell
 * lookup (images of cells in the 3^3 block of boxes around the box).  What the
 * levels >= 3 do not take (every image beyond that block, and the images of
 * level-2 cells whose level-1 father image does not touch the target's level-1
 * ancestor) enters the local expansions of FMM level 2 from all 64 level-2
 * cells, L_b(y) = sum_s sum_a (-1)^|a|/a! T_{a+b} M_a(s), with
 * T = D^lat(c_y - c_s) + sum of D(c_y - c_s - nL) over those block images n;
 * D^lat_g(d) = d^g(-F)(d), F = Ewald sum minus the 27 nearest images
 * (oracle_lattice).  Between level-2 cells these expansions converge much
 * faster than at the root or from level-1 sources.
 *
 * Derivatives D_g = d^g(-1/r) are evaluated from exact integer polynomials:
 * d^g (1/r) = P_g(x) / r^(2|g|+1) with P_{g+e_i} = r^2 dP_g/dx_i - (2|g|+1) x_i P_g.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_E_INVALID (-1)
#define OR_E_NOT_GRADED (-2)
#define OR_E_INCOMPLETE (-3)
#define OR_E_UNSUPPORTED (-4)
#define OR_E_NOMEM (-5)
#define OR_E_STATE (-7)

#define PMAX 10
#define NMI 286 /* C(PMAX+3, 3) */
#define MAXLEV 21

/* ------------------------------------------------------------------ */
/* multi-indices, graded by total degree                               */
/* ------------------------------------------------------------------ */
static int g_mi[NMI][3];
static int g_idx[PMAX + 2][PMAX + 2][PMAX + 2];
static double g_fact[PMAX + 2];
static int g_ready = 0;
/* numerator polynomials of d^g(1/r): sparse term lists */
typedef struct { double c; int e[3]; } term_t;
static term_t *g_terms[NMI];
static int g_nterms[NMI];

static int nmi_of(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

static void init_tables(void) {
  if (g_ready) return;
  int n = 0;
  for (int d = 0; d <= PMAX; ++d)
    for (int a = d; a >= 0; --a)
      for (int b = d - a; b >= 0; --b) {
        int c = d - a - b;
        g_mi[n][0] = a; g_mi[n][1] = b; g_mi[n][2] = c;
        g_idx[a][b][c] = n;
        ++n;
      }
  g_fact[0] = 1.0;
  for (int i = 1; i <= PMAX + 1; ++i) g_fact[i] = g_fact[i - 1] * i;

  /* dense polynomial workspace: coefficient of x^a y^b z^c */
  enum { D = PMAX + 3 };
  double *dense = (double *)calloc((size_t)NMI * D * D * D, sizeof(double));
#define PC(g, a, b, c) dense[(((size_t)(g) * D + (a)) * D + (b)) * D + (c)]
  PC(0, 0, 0, 0) = 1.0;
  for (int g = 1; g < NMI; ++g) {
    int ga[3] = {g_mi[g][0], g_mi[g][1], g_mi[g][2]};
    int i = ga[0] > 0 ? 0 : (ga[1] > 0 ? 1 : 2);
    int pa[3] = {ga[0], ga[1], ga[2]};
    pa[i] -= 1;
    int par = g_idx[pa[0]][pa[1]][pa[2]];
    int nd = pa[0] + pa[1] + pa[2];
    /* P_g = (x^2+y^2+z^2) dP/dx_i - (2 nd + 1) x_i P */
    for (int a = 0; a <= nd; ++a)
      for (int b = 0; a + b <= nd; ++b) {
        int c = nd - a - b;
        double v = PC(par, a, b, c);
        if (v == 0.0) continue;
        int e[3] = {a, b, c};
        if (e[i] > 0) {
          double dv = v * e[i];
          int f[3] = {a, b, c};
          f[i] -= 1;
          for (int k = 0; k < 3; ++k) {
            int h[3] = {f[0], f[1], f[2]};
            h[k] += 2;
            PC(g, h[0], h[1], h[2]) += dv;
          }
        }
        int h[3] = {a, b, c};
        h[i] += 1;
        PC(g, h[0], h[1], h[2]) -= (2.0 * nd + 1.0) * v;
      }
  }
  for (int g = 0; g < NMI; ++g) {
    int cnt = 0;
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b)
        for (int c = 0; c < D; ++c)
          if (PC(g, a, b, c) != 0.0) ++cnt;
    g_terms[g] = (term_t *)malloc(sizeof(term_t) * (cnt ? cnt : 1));
    g_nterms[g] = 0;
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b)
        for (int c = 0; c < D; ++c)
          if (PC(g, a, b, c) != 0.0) {
            term_t t;
            t.c = PC(g, a, b, c);
            t.e[0] = a; t.e[1] = b; t.e[2] = c;
            g_terms[g][g_nterms[g]++] = t;
          }
  }
#undef PC
  free(dense);
  g_ready = 1;
}

/* D_g(R) = d^g(-1/r) for all |g| <= n (G not included). */
static void derivs(int n, const double R[3], double *out) {
  double pw[3][PMAX + 3];
  for (int k = 0; k < 3; ++k) {
    pw[k][0] = 1.0;
    for (int e = 1; e < PMAX + 3; ++e) pw[k][e] = pw[k][e - 1] * R[k];
  }
  double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
  double r = sqrt(r2);
  double inv = 1.0 / r;
  double inv2 = inv * inv;
  double rp = inv; /* 1 / r^(2d+1) */
  int K = nmi_of(n);
  int deg = 0;
  for (int g = 0; g < K; ++g) {
    int d = g_mi[g][0] + g_mi[g][1] + g_mi[g][2];
    while (deg < d) { rp *= inv2; ++deg; }
    double s = 0.0;
    for (int t = 0; t < g_nterms[g]; ++t) {
      const term_t *tt = &g_terms[g][t];
      s += tt->c * pw[0][tt->e[0]] * pw[1][tt->e[1]] * pw[2][tt->e[2]];
    }
    out[g] = -s * rp;
  }
}

static double mono(const int *a, const double *x) {
  double v = 1.0;
  for (int k = 0; k < 3; ++k)
    for (int e = 0; e < a[k]; ++e) v *= x[k];
  return v;
}
static double mfact(const int *a) { return g_fact[a[0]] * g_fact[a[1]] * g_fact[a[2]]; }

/* ------------------------------------------------------------------ */
/* the four translation steps of Sec. 2, multi-index form              */
/* ------------------------------------------------------------------ */
/* Eq. eq:M2L: L_b = sum_{|a| <= p-|b|} (-1)^|a| / a! D_{a+b}(R) M_a, R = c_target - c_source;
   multipoles enter up to order pm (p, or p - 1 with the paper's cap of Sec. 2) */
static void op_m2l(int p, int pm, const double R[3], const double *M, double *L, double scale) {
  double D[NMI];
  derivs(p, R, D);
  int K = nmi_of(p);
  for (int b = 0; b < K; ++b) {
    const int *bb = g_mi[b];
    int nb = bb[0] + bb[1] + bb[2];
    double s = 0.0;
    for (int a = 0; a < K; ++a) {
      const int *aa = g_mi[a];
      int na = aa[0] + aa[1] + aa[2];
      if (na + nb > p || na > pm) continue;
      double sg = (na & 1) ? -1.0 : 1.0;
      s += sg / mfact(aa) * D[g_idx[aa[0] + bb[0]][aa[1] + bb[1]][aa[2] + bb[2]]] * M[a];
    }
    L[b] += scale * s;
  }
}

/* The lattice images at the root: Eq. eq:M2L with the lattice tensors in place
   of D_{a+b}(R). */
static void op_lattice(int p, int pm, const double *lat, const double *M, double *L) {
  int K = nmi_of(p);
  for (int b = 0; b < K; ++b) {
    const int *bb = g_mi[b];
    int nb = bb[0] + bb[1] + bb[2];
    double sum = 0.0;
    for (int a = 0; a < K; ++a) {
      const int *aa = g_mi[a];
      int na = aa[0] + aa[1] + aa[2];
      if (na + nb > p || na > pm) continue;
      double sg = (na & 1) ? -1.0 : 1.0;
      sum += sg / mfact(aa) * lat[g_idx[aa[0] + bb[0]][aa[1] + bb[1]][aa[2] + bb[2]]] * M[a];
    }
    L[b] += sum;
  }
}

/* Eq. eq:L2L: L'_b = sum_{|g| <= p-|b|} a^g / g! L_{b+g}, a = new centre - old centre */
static void op_l2l(int p, const double a[3], const double *L, double *Lout) {
  int K = nmi_of(p);
  for (int b = 0; b < K; ++b) {
    const int *bb = g_mi[b];
    int nb = bb[0] + bb[1] + bb[2];
    double s = 0.0;
    for (int g = 0; g < K; ++g) {
      const int *gg = g_mi[g];
      int ng = gg[0] + gg[1] + gg[2];
      if (ng + nb > p) continue;
      s += mono(gg, a) / mfact(gg) * L[g_idx[bb[0] + gg[0]][bb[1] + gg[1]][bb[2] + gg[2]]];
    }
    Lout[b] += s;
  }
}

/* local expansion evaluated at offset u from its centre: phi and a = -grad phi */
static void op_l2p(int p, const double u[3], const double *L, double *phi, double acc[3]) {
  int K = nmi_of(p);
  double f = 0.0, g[3] = {0, 0, 0};
  for (int b = 0; b < K; ++b) {
    const int *bb = g_mi[b];
    f += L[b] * mono(bb, u) / mfact(bb);
    for (int i = 0; i < 3; ++i) {
      if (bb[i] == 0) continue;
      int c[3] = {bb[0], bb[1], bb[2]};
      c[i] -= 1;
      g[i] += L[b] * mono(c, u) / mfact(c);
    }
  }
  *phi += f;
  for (int i = 0; i < 3; ++i) acc[i] -= g[i];
}

/* multipole (about its centre) evaluated at R = x - c: Taylor series of Sec. 2, multipoles up to
   order pm (the gradient terms need |a| + 1 <= p, so they never see order p) */
static void op_m2p(int p, int pm, const double R[3], const double *M, double *phi, double acc[3]) {
  double D[NMI];
  derivs(p, R, D);
  int K = nmi_of(p);
  double f = 0.0, g[3] = {0, 0, 0};
  for (int a = 0; a < K; ++a) {
    const int *aa = g_mi[a];
    int na = aa[0] + aa[1] + aa[2];
    if (na > pm) continue;
    double w = ((na & 1) ? -1.0 : 1.0) / mfact(aa) * M[a];
    f += w * D[a];
    if (na + 1 <= p)
      for (int i = 0; i < 3; ++i) {
        int c[3] = {aa[0], aa[1], aa[2]};
        c[i] += 1;
        g[i] += w * D[g_idx[c[0]][c[1]][c[2]]];
      }
  }
  *phi += f;
  for (int i = 0; i < 3; ++i) acc[i] -= g[i];
}

/* point mass: phi = -m/r, a = -m R / r^3 (G applied by the caller) */
static void op_p2p(const double R[3], double m, double *phi, double acc[3]) {
  double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
  double r = sqrt(r2);
  *phi -= m / r;
  double w = m / (r2 * r);
  for (int i = 0; i < 3; ++i) acc[i] -= w * R[i];
}

/* Eq. eq:M2M_general: M'_a = sum_{k <= a} C(a,k) (-t)^(a-k) M_k, t = new centre - old centre */
static void op_m2m(int p, const double t[3], const double *M, double *Mout) {
  int K = nmi_of(p);
  double mt[3] = {-t[0], -t[1], -t[2]};
  for (int a = 0; a < K; ++a) {
    const int *aa = g_mi[a];
    double s = 0.0;
    for (int k = 0; k < K; ++k) {
      const int *kk = g_mi[k];
      if (kk[0] > aa[0] || kk[1] > aa[1] || kk[2] > aa[2]) continue;
      int d[3] = {aa[0] - kk[0], aa[1] - kk[1], aa[2] - kk[2]};
      double binom = mfact(aa) / (mfact(kk) * mfact(d));
      s += binom * mono(d, mt) * M[k];
    }
    Mout[a] += s;
  }
}

/* ------------------------------------------------------------------ */
/* hash map: int64 key -> int64 value                                  */
/* ------------------------------------------------------------------ */
typedef struct { int64_t cap, n; int64_t *k, *v; } hmap;

static uint64_t hmix(uint64_t x) {
  x ^= x >> 33; x *= 0xff51afd7ed558ccdULL;
  x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ULL;
  x ^= x >> 33; return x;
}
static int hm_init(hmap *h, int64_t n) {
  int64_t cap = 16;
  while (cap < 2 * n + 16) cap <<= 1;
  h->cap = cap; h->n = 0;
  h->k = (int64_t *)malloc(sizeof(int64_t) * cap);
  h->v = (int64_t *)malloc(sizeof(int64_t) * cap);
  if (!h->k || !h->v) return OR_E_NOMEM;
  for (int64_t i = 0; i < cap; ++i) h->k[i] = -1;
  return OR_OK;
}
static void hm_free(hmap *h) { free(h->k); free(h->v); h->k = h->v = NULL; h->cap = h->n = 0; }
static int64_t hm_get(const hmap *h, int64_t key) {
  if (!h->cap) return -1;
  uint64_t m = (uint64_t)h->cap - 1, i = hmix((uint64_t)key) & m;
  while (h->k[i] != -1) {
    if (h->k[i] == key) return h->v[i];
    i = (i + 1) & m;
  }
  return -1;
}
/* insert if absent; returns the stored value */
static int64_t hm_put(hmap *h, int64_t key, int64_t val) {
  uint64_t m = (uint64_t)h->cap - 1, i = hmix((uint64_t)key) & m;
  while (h->k[i] != -1) {
    if (h->k[i] == key) return h->v[i];
    i = (i + 1) & m;
  }
  h->k[i] = key; h->v[i] = val; h->n++;
  return val;
}

static int64_t key3(int64_t i, int64_t j, int64_t k) { return (i << 42) | (j << 21) | k; }
static void unkey3(int64_t key, int64_t c[3]) {
  c[0] = key >> 42; c[1] = (key >> 21) & ((1 << 21) - 1); c[2] = key & ((1 << 21) - 1);
}

/* ------------------------------------------------------------------ */
/* oracle state                                                        */
/* ------------------------------------------------------------------ */
typedef struct {           /* FMM grid T_{j;f} (or a merged grid) at one level */
  hmap map;                /* cell key -> row */
  int64_t rows;
  int64_t *keys;           /* [rows] */
  double *coef;            /* [rows][K] */
} grid_t;

typedef struct {
  int built;
  grid_t *g;               /* g[f] for f = 1 .. j-1 (index f) */
  double *leafmass;        /* [ncell(j)] masses of level-j leaves at last rebuild */
} tree_t;

typedef struct oracle_state {
  int levelmin, levelmax, p, K;
  int pm;                  /* highest multipole order used by M2L/M2P: p, or p - 1 with the cap */
  double cself;            /* self-potential constant (unit cube), 0 when the term is off */
  double G, boxlen;
  int64_t ncell[MAXLEV], off[MAXLEV + 1];
  int32_t *ijk;            /* flat [N][3] */
  uint8_t *refined;        /* flat [N] */
  hmap cellmap[MAXLEV];    /* level -> key -> flat index (AMR levels only) */
  tree_t tree[MAXLEV];
  int merged_all;          /* evaluate with per-source sums over all trees (pin P10) */
  int periodic;            /* torus box with a neutralising background */
  double *lat;             /* [8][7^3][K] level-2 far operators by target octant and offset (periodic) */
} oracle_state;

static double csize(const oracle_state *s, int lev) { return s->boxlen / (double)(1LL << lev); }
static void centre(const oracle_state *s, int lev, const int64_t c[3], double x[3]) {
  double h = csize(s, lev);
  for (int k = 0; k < 3; ++k) x[k] = ((double)c[k] + 0.5) * h;
}

/* cell existence: -2 = outside box, -1 = absent, else flat index; virtual levels return -3 */
#define CELL_OUT (-2)
#define CELL_ABSENT (-1)
#define CELL_VIRTUAL (-3)
/* periodic boxes: the cell of the torus that c (any integer coordinates) lands on */
static void wrap3(const oracle_state *s, int lev, const int64_t c[3], int64_t w[3]) {
  int64_t n = 1LL << lev;
  for (int k = 0; k < 3; ++k) w[k] = s->periodic ? ((c[k] % n) + n) % n : c[k];
}
static int64_t cell_lookup(const oracle_state *s, int lev, const int64_t c0[3]) {
  int64_t n = 1LL << lev, c[3];
  wrap3(s, lev, c0, c);
  for (int k = 0; k < 3; ++k)
    if (c[k] < 0 || c[k] >= n) return CELL_OUT;
  if (lev < s->levelmin) return CELL_VIRTUAL;
  if (lev > s->levelmax) return CELL_ABSENT;
  int64_t v = hm_get(&s->cellmap[lev], key3(c[0], c[1], c[2]));
  return v < 0 ? CELL_ABSENT : v;
}
static int is_refined_cell(const oracle_state *s, int64_t idx) {
  return idx == CELL_VIRTUAL || (idx >= 0 && s->refined[idx]);
}

static void grid_free(grid_t *g) {
  hm_free(&g->map);
  free(g->keys); free(g->coef);
  memset(g, 0, sizeof(*g));
}
static void tree_free(oracle_state *s, int j) {
  tree_t *t = &s->tree[j];
  if (t->g) {
    for (int f = 1; f < j; ++f) grid_free(&t->g[f]);
    free(t->g);
  }
  free(t->leafmass);
  memset(t, 0, sizeof(*t));
}

void oracle_destroy(oracle_state *s) {
  if (!s) return;
  for (int l = 0; l < MAXLEV; ++l) {
    tree_free(s, l);
    hm_free(&s->cellmap[l]);
  }
  free(s->ijk); free(s->refined); free(s->lat);
  free(s);
}

/* strong grading: a refined level-l cell needs the 27 neighbours of its father
   refined (clipped to the box, or wrapped around a periodic one) */
static int check_grading(const oracle_state *s) {
  for (int l = s->levelmin + 1; l <= s->levelmax; ++l)
    for (int64_t i = s->off[l]; i < s->off[l + 1]; ++i) {
      if (!s->refined[i]) continue;
      const int32_t *c = &s->ijk[3 * i];
      for (int e = 0; e < 27; ++e) {
        int64_t q[3] = {c[0] / 2 + e % 3 - 1, c[1] / 2 + (e / 3) % 3 - 1, c[2] / 2 + e / 9 - 1};
        int64_t qi = cell_lookup(s, l - 1, q);
        if (qi == CELL_OUT) continue;
        if (!is_refined_cell(s, qi)) return OR_E_NOT_GRADED;
      }
    }
  return OR_OK;
}

/* Build the AMR cell maps and check completeness and the strong grading rule. */
int oracle_create(int levelmin, int levelmax, const int64_t *ncell, const int32_t *ijk,
                  const uint8_t *refined, int p, double G, double boxlen, oracle_state **out) {
  init_tables();
  *out = NULL;
  if (levelmin < 1 || levelmax < levelmin || levelmax >= MAXLEV - 1) return OR_E_INVALID;
  if (p < 1 || p > PMAX - 1) return OR_E_UNSUPPORTED;
  oracle_state *s = (oracle_state *)calloc(1, sizeof(oracle_state));
  if (!s) return OR_E_NOMEM;
  s->levelmin = levelmin; s->levelmax = levelmax; s->p = p; s->K = nmi_of(p);
  s->pm = p; s->cself = 0.0;
  s->G = G; s->boxlen = boxlen;
  int64_t N = 0;
  for (int l = levelmin; l <= levelmax; ++l) {
    s->ncell[l] = ncell[l - levelmin];
    s->off[l] = N;
    N += s->ncell[l];
  }
  s->off[levelmax + 1] = N;
  s->ijk = (int32_t *)malloc(sizeof(int32_t) * 3 * (N ? N : 1));
  s->refined = (uint8_t *)malloc(N ? N : 1);
  memcpy(s->ijk, ijk, sizeof(int32_t) * 3 * N);
  memcpy(s->refined, refined, N);
  int rc = OR_OK;
  if (s->ncell[levelmin] != (1LL << (3 * levelmin))) rc = OR_E_INCOMPLETE;
  for (int l = levelmin; l <= levelmax && rc == OR_OK; ++l) {
    if (hm_init(&s->cellmap[l], s->ncell[l]) != OR_OK) { rc = OR_E_NOMEM; break; }
    int64_t n = 1LL << l;
    for (int64_t i = s->off[l]; i < s->off[l + 1]; ++i) {
      const int32_t *c = &s->ijk[3 * i];
      if (c[0] < 0 || c[0] >= n || c[1] < 0 || c[1] >= n || c[2] < 0 || c[2] >= n) { rc = OR_E_INVALID; break; }
      int64_t k = key3(c[0], c[1], c[2]);
      if (hm_put(&s->cellmap[l], k, i) != i) { rc = OR_E_INVALID; break; }
    }
  }
  /* completeness: children of refined cells exist; every cell has a refined father */
  for (int l = levelmin; l <= levelmax && rc == OR_OK; ++l) {
    int64_t nref = 0;
    for (int64_t i = s->off[l]; i < s->off[l + 1]; ++i) {
      if (!s->refined[i]) continue;
      ++nref;
      if (l == levelmax) { rc = OR_E_INCOMPLETE; break; }
      const int32_t *c = &s->ijk[3 * i];
      for (int o = 0; o < 8; ++o) {
        int64_t ch[3] = {2LL * c[0] + (o & 1), 2LL * c[1] + ((o >> 1) & 1), 2LL * c[2] + ((o >> 2) & 1)};
        if (cell_lookup(s, l + 1, ch) < 0) { rc = OR_E_INCOMPLETE; break; }
      }
    }
    if (rc == OR_OK && l < levelmax && s->ncell[l + 1] != 8 * nref) rc = OR_E_INCOMPLETE;
  }
  if (rc == OR_OK) rc = check_grading(s);
  if (rc != OR_OK) { oracle_destroy(s); return rc; }
  *out = s;
  return OR_OK;
}

void oracle_set_merged_all(oracle_state *s, int on) { s->merged_all = on; }

/*
 * Self-potential constant C = integral over the unit cube centred at the
 * origin of 1/|r| (reading R11: a leaf's own mass as a uniform cube, whose
 * potential at its centre is -G m C / h).  C is 8 times the integral over the
 * octant [0, 1/2]^3.  There the z-integral is elementary,
 *   int_0^{1/2} dz / sqrt(rho^2 + z^2) = asinh(1 / (2 rho)),  rho^2 = x^2 + y^2,
 * and in polar coordinates over the square [0, 1/2]^2 (two symmetric halves,
 * 0 <= theta <= pi/4, rho up to 1 / (2 cos theta)) so is the rho-integral:
 *   int rho asinh(1 / (2 rho)) drho = F(rho) = rho^2/2 asinh(1/(2 rho)) + sqrt(rho^2 + 1/4)/4,
 * F(0) = 1/8.  What is left, C = 16 int_0^{pi/4} [F(1/(2 cos theta)) - 1/8] dtheta,
 * has a smooth integrand and is summed with a composite Simpson rule.
 */
static double self_F(double rho) { return 0.5 * rho * rho * asinh(0.5 / rho) + 0.25 * sqrt(rho * rho + 0.25); }
double oracle_self_constant(void) {
  const int n = 4096; /* even */
  const double b = atan(1.0), h = b / n;
  double sum = 0.0;
  for (int i = 0; i <= n; ++i) {
    double t = i * h;
    double f = self_F(0.5 / cos(t)) - 0.125;
    sum += f * (i == 0 || i == n ? 1.0 : (i & 1) ? 4.0 : 2.0);
  }
  return 16.0 * sum * h / 3.0;
}

/* Model options: AFMM-style paper cap (multipoles to order p - 1, Sec. 2 with
   reading R1) and the optional self-potential term (reading R11). */
int oracle_set_options(oracle_state *s, int quad_cap, int self_potential) {
  if (!s) return OR_E_INVALID;
  s->pm = quad_cap ? s->p - 1 : s->p;
  s->cself = self_potential ? oracle_self_constant() : 0.0;
  return OR_OK;
}

static uint64_t morton3(int64_t x, int64_t y, int64_t z) {
  uint64_t k = 0;
  for (int b = 0; b < 21; ++b) {
    k |= (uint64_t)((x >> b) & 1) << (3 * b);
    k |= (uint64_t)((y >> b) & 1) << (3 * b + 1);
    k |= (uint64_t)((z >> b) & 1) << (3 * b + 2);
  }
  return k;
}
typedef struct { uint64_t m; int64_t i; } mrec;
static int cmp_mrec(const void *a, const void *b) {
  uint64_t x = ((const mrec *)a)->m, y = ((const mrec *)b)->m;
  return x < y ? -1 : (x > y);
}

/*
 * Alg. 2 (BuildTree + Upward + CenterShift) for tree j.  The moments are taken
 * about each FMM cell's geometric centre directly from their definition, so
 * CenterShift is the identity here.
 */
static int build_tree(oracle_state *s, int j, const double *mass) {
  tree_free(s, j);
  tree_t *t = &s->tree[j];
  int K = s->K;
  int64_t n = s->ncell[j], o = s->off[j];
  t->leafmass = (double *)calloc(n ? n : 1, sizeof(double));
  t->g = (grid_t *)calloc(j, sizeof(grid_t));
  if (!t->leafmass || !t->g) return OR_E_NOMEM;
  int64_t nl = 0;
  for (int64_t i = 0; i < n; ++i)
    if (!s->refined[o + i]) { t->leafmass[i] = mass[o + i]; ++nl; }
  mrec *rec = (mrec *)malloc(sizeof(mrec) * (nl ? nl : 1));
  nl = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (s->refined[o + i]) continue;
    const int32_t *c = &s->ijk[3 * (o + i)];
    rec[nl].m = morton3(c[0], c[1], c[2]);
    rec[nl].i = i;
    ++nl;
  }
  qsort(rec, nl, sizeof(mrec), cmp_mrec);
  for (int f = 1; f <= j - 1; ++f) {
    grid_t *g = &t->g[f];
    int sh = 3 * (j - f);
    /* runs of equal ancestors are contiguous in Morton order */
    int64_t runs = 0;
    for (int64_t a = 0; a < nl; ++a)
      if (a == 0 || (rec[a].m >> sh) != (rec[a - 1].m >> sh)) ++runs;
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (runs + 1));
    runs = 0;
    for (int64_t a = 0; a < nl; ++a)
      if (a == 0 || (rec[a].m >> sh) != (rec[a - 1].m >> sh)) start[runs++] = a;
    start[runs] = nl;
    g->rows = runs;
    g->keys = (int64_t *)malloc(sizeof(int64_t) * (runs ? runs : 1));
    g->coef = (double *)calloc((size_t)(runs ? runs : 1) * K, sizeof(double));
    if (hm_init(&g->map, runs) != OR_OK || !g->keys || !g->coef) { free(start); free(rec); return OR_E_NOMEM; }
    int shl = j - f;
    for (int64_t r = 0; r < runs; ++r) {
      const int32_t *c = &s->ijk[3 * (o + rec[start[r]].i)];
      int64_t a3[3] = {c[0] >> shl, c[1] >> shl, c[2] >> shl};
      g->keys[r] = key3(a3[0], a3[1], a3[2]);
      hm_put(&g->map, g->keys[r], r);
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < runs; ++r) {
      int64_t a3[3];
      unkey3(g->keys[r], a3);
      double cy[3];
      centre(s, f, a3, cy);
      double *M = &g->coef[r * K];
      for (int64_t a = start[r]; a < start[r + 1]; ++a) {
        int64_t li = rec[a].i;
        const int32_t *c = &s->ijk[3 * (o + li)];
        int64_t c3[3] = {c[0], c[1], c[2]};
        double x[3], d[3];
        centre(s, j, c3, x);
        for (int k = 0; k < 3; ++k) d[k] = x[k] - cy[k];
        double m = t->leafmass[li];
        for (int q = 0; q < K; ++q) M[q] += m * mono(g_mi[q], d);
      }
    }
    free(start);
  }
  free(rec);
  t->built = 1;
  return OR_OK;
}

/* RebuildTree(l): trees j = l .. levelmax from the given flat masses. */
int oracle_rebuild(oracle_state *s, int level, const double *mass) {
  if (level < s->levelmin || level > s->levelmax) return OR_E_INVALID;
  for (int j = level; j <= s->levelmax; ++j) {
    int rc = build_tree(s, j, mass);
    if (rc) return rc;
  }
  return OR_OK;
}

/* sum of grids g[f] of trees jlo..jhi (merged tree ~T at one FMM level) */
static int merge_grids(oracle_state *s, int jlo, int jhi, int f, grid_t *out) {
  int K = s->K;
  memset(out, 0, sizeof(*out));
  int64_t cap = 0;
  for (int j = jlo; j <= jhi; ++j)
    if (f <= j - 1) cap += s->tree[j].g[f].rows;
  if (hm_init(&out->map, cap) != OR_OK) return OR_E_NOMEM;
  out->keys = (int64_t *)malloc(sizeof(int64_t) * (cap ? cap : 1));
  out->coef = (double *)calloc((size_t)(cap ? cap : 1) * K, sizeof(double));
  if (!out->keys || !out->coef) return OR_E_NOMEM;
  for (int j = jlo; j <= jhi; ++j) {
    if (f > j - 1) continue;
    grid_t *g = &s->tree[j].g[f];
    for (int64_t r = 0; r < g->rows; ++r) {
      int64_t row = hm_put(&out->map, g->keys[r], out->rows);
      if (row == out->rows) out->keys[out->rows++] = g->keys[r];
      for (int q = 0; q < K; ++q) out->coef[row * K + q] += g->coef[r * K + q];
    }
  }
  return OR_OK;
}

static const double *grid_row(const grid_t *g, const int64_t c[3], int K) {
  if (!g || !g->rows) return NULL;
  int64_t r = hm_get(&g->map, key3(c[0], c[1], c[2]));
  return r < 0 ? NULL : &g->coef[r * K];
}

/* evaluation context for one target level */
typedef struct {
  int l;
  grid_t mrg[MAXLEV];      /* ~T_{l+1;f}, f = 1..l      */
  grid_t all[MAXLEV];      /* sum of every tree at f (merged_all mode) */
  grid_t Lg[MAXLEV];       /* L_{l;f} for the needed FMM cells, f = 2..l-1 */
} evalctx;

static void ctx_free(evalctx *c) {
  for (int f = 0; f < MAXLEV; ++f) { grid_free(&c->mrg[f]); grid_free(&c->all[f]); grid_free(&c->Lg[f]); }
}

static double leafmass_of(const oracle_state *s, int lev, int64_t idx) {
  return s->tree[lev].leafmass[idx - s->off[lev]];
}

/*
 * Sources of the interaction list of a target at level f (Sec. 2): level-(f-1)
 * cells of the 6^3 block around the father's oct, i.e. children of the 27
 * neighbours of the grandfather, minus the 27 cells touching the father.
 * Calls back with each in-box source; returns OR_E_NOT_GRADED if one is absent.
 */
typedef void (*src_cb)(void *u, int lev, const int64_t sc[3], int64_t idx);
static int foreach_il(const oracle_state *s, int f, const int64_t y[3], src_cb cb, void *u) {
  if (f < 2) return OR_OK;
  int64_t F[3] = {y[0] >> 1, y[1] >> 1, y[2] >> 1};
  int64_t Gc[3] = {F[0] >> 1, F[1] >> 1, F[2] >> 1};
  for (int e = 0; e < 27; ++e) {
    int64_t Q[3] = {Gc[0] + e % 3 - 1, Gc[1] + (e / 3) % 3 - 1, Gc[2] + e / 9 - 1};
    if (f - 2 >= 0 && !s->periodic) {
      int64_t nq = 1LL << (f - 2);
      if (Q[0] < 0 || Q[0] >= nq || Q[1] < 0 || Q[1] >= nq || Q[2] < 0 || Q[2] >= nq) continue;
    }
    for (int o = 0; o < 8; ++o) {
      int64_t sc[3] = {2 * Q[0] + (o & 1), 2 * Q[1] + ((o >> 1) & 1), 2 * Q[2] + ((o >> 2) & 1)};
      int64_t dx = llabs(sc[0] - F[0]), dy = llabs(sc[1] - F[1]), dz = llabs(sc[2] - F[2]);
      int64_t dm = dx > dy ? dx : dy;
      dm = dm > dz ? dm : dz;
      if (dm <= 1) continue;
      int64_t idx = cell_lookup(s, f - 1, sc);
      if (idx == CELL_OUT) continue;
      if (idx == CELL_ABSENT) return OR_E_NOT_GRADED;
      cb(u, f - 1, sc, idx);
    }
  }
  return OR_OK;
}

typedef struct {
  const oracle_state *s;
  const evalctx *c;
  double cy[3];
  double *L;
  int f;        /* target FMM level */
} m2l_u;

static void m2l_src(void *uu, int lev, const int64_t sc0[3], int64_t idx) {
  m2l_u *u = (m2l_u *)uu;
  const oracle_state *s = u->s;
  int K = s->K, l = u->c->l;
  double cs[3], R[3];
  int64_t sc[3];
  centre(s, lev, sc0, cs);      /* the image's own position */
  wrap3(s, lev, sc0, sc);       /* the cell it is an image of */
  for (int k = 0; k < 3; ++k) R[k] = u->cy[k] - cs[k];
  if (s->merged_all) {
    /* one source multipole: sum over every tree (and the leaf mass) */
    double M[NMI];
    memset(M, 0, sizeof(double) * K);
    if (idx >= 0 && !s->refined[idx]) M[0] += leafmass_of(s, lev, idx);
    const double *A = grid_row(&u->c->all[lev], sc, K);
    if (A) for (int q = 0; q < K; ++q) M[q] += A[q];
    op_m2l(s->p, s->pm, R, M, u->L, 1.0);
    return;
  }
  /* Alg. 3: trees j = max(lmin, f-1) .. l one by one, then the merged tree */
  int jlo = s->levelmin > lev ? s->levelmin : lev;
  for (int j = jlo; j <= l; ++j) {
    if (j == lev) {
      if (idx >= 0 && !s->refined[idx]) {
        double M[NMI];
        memset(M, 0, sizeof(double) * K);
        M[0] = leafmass_of(s, lev, idx);
        op_m2l(s->p, s->pm, R, M, u->L, 1.0);
      }
      continue;
    }
    const double *M = grid_row(&s->tree[j].g[lev], sc, K);
    if (M) op_m2l(s->p, s->pm, R, M, u->L, 1.0);
  }
  if (l < s->levelmax) {
    const double *M = grid_row(&u->c->mrg[lev], sc, K);
    if (M) op_m2l(s->p, s->pm, R, M, u->L, 1.0);
  }
}

typedef struct {
  const oracle_state *s;
  const evalctx *c;
  double x[3];
  double phi, acc[3];
} m2p_u;

/* intermediate field of a level-l target: one level-(l-1) source of its list */
static void m2p_src(void *uu, int lev, const int64_t sc0[3], int64_t idx) {
  m2p_u *u = (m2p_u *)uu;
  const oracle_state *s = u->s;
  int K = s->K, l = u->c->l;
  double cs[3], R[3];
  int64_t sc[3];
  centre(s, lev, sc0, cs);
  wrap3(s, lev, sc0, sc);
  for (int k = 0; k < 3; ++k) R[k] = u->x[k] - cs[k];
  if (idx >= 0 && !s->refined[idx]) {          /* level-(l-1) leaf: P2P (brown dots) */
    op_p2p(R, leafmass_of(s, lev, idx), &u->phi, u->acc);
    return;
  }
  if (s->merged_all) {
    const double *A = grid_row(&u->c->all[lev], sc, K);
    if (A) op_m2p(s->p, s->pm, R, A, &u->phi, u->acc);
    return;
  }
  const double *M = grid_row(&s->tree[l].g[lev], sc, K);       /* T_{l;l-1} (blue dots) */
  if (M) op_m2p(s->p, s->pm, R, M, &u->phi, u->acc);
  if (l < s->levelmax) {
    const double *Mm = grid_row(&u->c->mrg[lev], sc, K);       /* ~T_{l+1;l-1} (green dots) */
    if (Mm) op_m2p(s->p, s->pm, R, Mm, &u->phi, u->acc);
  }
}

static int64_t cheb(const int64_t a[3], const int64_t b[3]) {
  int64_t m = 0;
  for (int k = 0; k < 3; ++k) {
    int64_t d = llabs(a[k] - b[k]);
    if (d > m) m = d;
  }
  return m;
}

/* far + intermediate + near + nearest for one level-l leaf (Alg. 4, Sec. 3.2) */
static int eval_leaf(const oracle_state *s, const evalctx *c, int64_t flat, double *phi, double acc[3],
                     double part[4][4]) {
  int l = c->l, K = s->K;
  const int32_t *ci = &s->ijk[3 * flat];
  int64_t cc[3] = {ci[0], ci[1], ci[2]};
  double x[3];
  centre(s, l, cc, x);
  int64_t F[3] = {cc[0] >> 1, cc[1] >> 1, cc[2] >> 1};
  double p_far = 0, a_far[3] = {0, 0, 0};
  /* far field: ShiftLocal of L_{l;l-1} to the cell */
  if (l - 1 >= (s->periodic ? 0 : 2)) {
    const double *L = grid_row(&c->Lg[l - 1], F, K);
    if (!L) return OR_E_STATE;
    double cF[3], u[3];
    centre(s, l - 1, F, cF);
    for (int k = 0; k < 3; ++k) u[k] = x[k] - cF[k];
    op_l2p(s->p, u, L, &p_far, a_far);
  }
  /* intermediate field */
  m2p_u mu;
  mu.s = s; mu.c = c;
  memcpy(mu.x, x, sizeof(x));
  mu.phi = 0; mu.acc[0] = mu.acc[1] = mu.acc[2] = 0;
  int rc = foreach_il(s, l, cc, m2p_src, &mu);
  if (rc) return rc;
  /* near and nearest fields */
  double p_near = 0, a_near[3] = {0, 0, 0};
  double p_nst = 0, a_nst[3] = {0, 0, 0};
  for (int e = 0; e < 27; ++e) {
    int64_t q[3] = {F[0] + e % 3 - 1, F[1] + (e / 3) % 3 - 1, F[2] + e / 9 - 1};
    int64_t qi = cell_lookup(s, l - 1, q);
    if (qi == CELL_OUT) continue;
    if (qi == CELL_ABSENT) return OR_E_NOT_GRADED;
    double R[3], cq[3];
    if (!is_refined_cell(s, qi)) {                 /* level-(l-1) leaf: P2P */
      centre(s, l - 1, q, cq);
      for (int k = 0; k < 3; ++k) R[k] = x[k] - cq[k];
      op_p2p(R, leafmass_of(s, l - 1, qi), &p_near, a_near);
      continue;
    }
    for (int o = 0; o < 8; ++o) {
      int64_t n3[3] = {2 * q[0] + (o & 1), 2 * q[1] + ((o >> 1) & 1), 2 * q[2] + ((o >> 2) & 1)};
      if (n3[0] == cc[0] && n3[1] == cc[1] && n3[2] == cc[2]) continue;   /* no self term */
      int64_t ni = cell_lookup(s, l, n3);
      if (ni < 0) return OR_E_NOT_GRADED;
      double cn[3];
      centre(s, l, n3, cn);
      for (int k = 0; k < 3; ++k) R[k] = x[k] - cn[k];
      if (!s->refined[ni]) {                          /* level-l leaf: P2P */
        op_p2p(R, leafmass_of(s, l, ni), &p_near, a_near);
      } else if (cheb(n3, cc) <= 1) {                 /* nearest field: its 8 children */
        for (int o2 = 0; o2 < 8; ++o2) {
          int64_t k3[3] = {2 * n3[0] + (o2 & 1), 2 * n3[1] + ((o2 >> 1) & 1), 2 * n3[2] + ((o2 >> 2) & 1)};
          int64_t ki = cell_lookup(s, l + 1, k3);
          if (ki < 0) return OR_E_INCOMPLETE;
          if (s->refined[ki]) return OR_E_NOT_GRADED;
          double ck[3], Rk[3];
          centre(s, l + 1, k3, ck);
          for (int k = 0; k < 3; ++k) Rk[k] = x[k] - ck[k];
          op_p2p(Rk, leafmass_of(s, l + 1, ki), &p_nst, a_nst);
        }
      } else {                                        /* M2P from ~T_{l+1;l} */
        int64_t w3[3];
        wrap3(s, l, n3, w3);
        const double *M = s->merged_all ? grid_row(&c->all[l], w3, K) : grid_row(&c->mrg[l], w3, K);
        if (!M) return OR_E_STATE;
        op_m2p(s->p, s->pm, R, M, &p_near, a_near);
      }
    }
  }
  /* optional self term: the leaf's own mass as a uniform cube (reading R11) */
  if (s->cself != 0.0) p_near -= s->cself * leafmass_of(s, l, flat) / csize(s, l);
  double G = s->G;
  *phi = G * (p_far + mu.phi + p_near + p_nst);
  for (int k = 0; k < 3; ++k) acc[k] = G * (a_far[k] + mu.acc[k] + a_near[k] + a_nst[k]);
  if (part) {
    part[0][0] = G * p_far; part[1][0] = G * mu.phi; part[2][0] = G * p_near; part[3][0] = G * p_nst;
    for (int k = 0; k < 3; ++k) {
      part[0][k + 1] = G * a_far[k]; part[1][k + 1] = G * mu.acc[k];
      part[2][k + 1] = G * a_near[k]; part[3][k + 1] = G * a_nst[k];
    }
  }
  return OR_OK;
}

/* Periodic boxes: the level-2 far operator, from every level-2 cell s
   (multipoles of the same trees as M2L reads) into the level-2 target y. */
static void lattice_m2l(const oracle_state *s, const evalctx *c, const int64_t y[3], double *L) {
  int K = s->K, l = c->l;
  for (int64_t a = 0; a < 4; ++a)
    for (int64_t b = 0; b < 4; ++b)
      for (int64_t d = 0; d < 4; ++d) {
        const int64_t sc[3] = {a, b, d};
        double M[NMI];
        memset(M, 0, sizeof(double) * K);
        if (s->merged_all) {
          const double *A = grid_row(&c->all[2], sc, K);
          if (A) for (int q = 0; q < K; ++q) M[q] += A[q];
        } else {
          for (int j = s->levelmin; j <= l; ++j) {
            const double *A = grid_row(&s->tree[j].g[2], sc, K);
            if (A) for (int q = 0; q < K; ++q) M[q] += A[q];
          }
          if (l < s->levelmax) {
            const double *A = grid_row(&c->mrg[2], sc, K);
            if (A) for (int q = 0; q < K; ++q) M[q] += A[q];
          }
        }
        int di = (int)((a - y[0] + 3) + 7 * (b - y[1] + 3) + 49 * (d - y[2] + 3));
        int oy = (int)((y[0] & 1) | (y[1] & 1) << 1 | (y[2] & 1) << 2);
        op_lattice(s->p, s->pm, &s->lat[((size_t)oy * 343 + di) * K], M, L);
      }
}

/*
 * Evaluate level-l leaves `targets` (flat indices) with the current trees:
 * Alg. 1 from RebuildMergedTree on (merged tree, L = 0, Alg. 3, Alg. 4).
 * part (optional) receives [ntarget][4 fields][phi, ax, ay, az].
 */
int oracle_eval(oracle_state *s, int l, int64_t ntarget, const int64_t *targets, double *phi, double *acc,
                double *part) {
  if (l < s->levelmin || l > s->levelmax) return OR_E_INVALID;
  for (int j = s->levelmin; j <= s->levelmax; ++j)
    if (!s->tree[j].built) return OR_E_STATE;
  int K = s->K;
  for (int64_t t = 0; t < ntarget; ++t) {
    int64_t i = targets[t];
    if (i < s->off[l] || i >= s->off[l + 1] || s->refined[i]) return OR_E_INVALID;
  }
  evalctx *c = (evalctx *)calloc(1, sizeof(evalctx));
  c->l = l;
  int rc = OR_OK;
  /* RebuildMergedTree: ~T_{l+1} = Merge(T_{l+1} .. T_lmax) at FMM levels 1..l */
  if (l < s->levelmax)
    for (int f = 1; f <= l && rc == OR_OK; ++f) rc = merge_grids(s, l + 1, s->levelmax, f, &c->mrg[f]);
  if (s->merged_all)
    for (int f = 1; f <= s->levelmax - 1 && rc == OR_OK; ++f)
      rc = merge_grids(s, s->levelmin, s->levelmax, f, &c->all[f]);
  /* needed FMM cells of T_l: ancestors of the targets at levels 2 .. l-1 */
  for (int f = 2; f <= l - 1 && rc == OR_OK; ++f) {
    grid_t *g = &c->Lg[f];
    if (hm_init(&g->map, ntarget) != OR_OK) { rc = OR_E_NOMEM; break; }
    g->keys = (int64_t *)malloc(sizeof(int64_t) * (ntarget ? ntarget : 1));
    for (int64_t t = 0; t < ntarget; ++t) {
      const int32_t *ci = &s->ijk[3 * targets[t]];
      int sh = l - f;
      int64_t k = key3(ci[0] >> sh, ci[1] >> sh, ci[2] >> sh);
      int64_t row = hm_put(&g->map, k, g->rows);
      if (row == g->rows) g->keys[g->rows++] = k;
    }
    g->coef = (double *)calloc((size_t)(g->rows ? g->rows : 1) * K, sizeof(double));
  }
  /* Alg. 3 MultipoleToLocal, level by level from f = 2 (L = 0 at f = 1) */
  for (int f = 2; f <= l - 1 && rc == OR_OK; ++f) {
    grid_t *g = &c->Lg[f];
    int err = OR_OK;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < g->rows; ++r) {
      int64_t y[3];
      unkey3(g->keys[r], y);
      double *L = &g->coef[r * K];
      if (f == 2 && s->periodic) lattice_m2l(s, c, y, L);
      if (f - 1 >= 2) {
        int64_t Fc[3] = {y[0] >> 1, y[1] >> 1, y[2] >> 1};
        const double *LF = grid_row(&c->Lg[f - 1], Fc, K);
        double cy[3], cF[3], a[3];
        centre(s, f, y, cy);
        centre(s, f - 1, Fc, cF);
        for (int k = 0; k < 3; ++k) a[k] = cy[k] - cF[k];
        if (LF) op_l2l(s->p, a, LF, L);
      }
      m2l_u u;
      u.s = s; u.c = c; u.L = L; u.f = f;
      centre(s, f, y, u.cy);
      /* periodic: the level-1 sources of level 2 are part of the level-2 far operator */
      int e2 = (f == 2 && s->periodic) ? OR_OK : foreach_il(s, f, y, m2l_src, &u);
      if (e2) {
#pragma omp critical
        err = e2;
      }
    }
    rc = err;
  }
  /* Alg. 4 PotentialEvaluation at each target leaf */
  if (rc == OR_OK) {
    int err = OR_OK;
#pragma omp parallel for schedule(dynamic, 32)
    for (int64_t t = 0; t < ntarget; ++t) {
      double pt[4][4];
      int e2 = eval_leaf(s, c, targets[t], &phi[t], &acc[3 * t], part ? pt : NULL);
      if (e2) {
#pragma omp critical
        err = e2;
      } else if (part) {
        memcpy(&part[16 * t], pt, sizeof(pt));
      }
    }
    rc = err;
  }
  ctx_free(c);
  free(c);
  return rc;
}

/*
 * Alg. 1 FMM Solve(l, icount): rebuild trees j >= l when l == levelmin or
 * icount > 1, then evaluate every level-l leaf.  phi/acc are flat arrays over
 * all cells; only level-l leaves are written.
 */
int oracle_solve(oracle_state *s, int l, int icount, const double *mass, double *phi, double *acc) {
  if (l < s->levelmin || l > s->levelmax) return OR_E_INVALID;
  if (l == s->levelmin || icount > 1) {
    int rc = oracle_rebuild(s, l, mass);
    if (rc) return rc;
  }
  int64_t n = 0;
  for (int64_t i = s->off[l]; i < s->off[l + 1]; ++i) n += !s->refined[i];
  int64_t *tg = (int64_t *)malloc(sizeof(int64_t) * (n ? n : 1));
  n = 0;
  for (int64_t i = s->off[l]; i < s->off[l + 1]; ++i)
    if (!s->refined[i]) tg[n++] = i;
  double *ph = (double *)malloc(sizeof(double) * (n ? n : 1));
  double *ac = (double *)malloc(sizeof(double) * 3 * (n ? n : 1));
  int rc = oracle_eval(s, l, n, tg, ph, ac, NULL);
  if (rc == OR_OK)
    for (int64_t t = 0; t < n; ++t) {
      phi[tg[t]] = ph[t];
      for (int k = 0; k < 3; ++k) acc[3 * tg[t] + k] = ac[3 * t + k];
    }
  free(tg); free(ph); free(ac);
  return rc;
}

/* Synchronous solve of every level (all trees fresh): the full-solve reference. */
int oracle_solve_all(oracle_state *s, const double *mass, double *phi, double *acc) {
  int rc = oracle_rebuild(s, s->levelmin, mass);
  for (int l = s->levelmin; l <= s->levelmax && rc == OR_OK; ++l) {
    int64_t n = 0;
    for (int64_t i = s->off[l]; i < s->off[l + 1]; ++i) n += !s->refined[i];
    int64_t *tg = (int64_t *)malloc(sizeof(int64_t) * (n ? n : 1));
    double *ph = (double *)malloc(sizeof(double) * (n ? n : 1));
    double *ac = (double *)malloc(sizeof(double) * 3 * (n ? n : 1));
    n = 0;
    for (int64_t i = s->off[l]; i < s->off[l + 1]; ++i)
      if (!s->refined[i]) tg[n++] = i;
    rc = oracle_eval(s, l, n, tg, ph, ac, NULL);
    if (rc == OR_OK)
      for (int64_t t = 0; t < n; ++t) {
        phi[tg[t]] = ph[t];
        for (int k = 0; k < 3; ++k) acc[3 * tg[t] + k] = ac[3 * t + k];
      }
    free(tg); free(ph); free(ac);
  }
  return rc;
}

/* ------------------------------------------------------------------ */
/* O(N^2) direct sum over point masses at cell centres                 */
/* ------------------------------------------------------------------ */
int oracle_direct(int64_t nsrc, const double *xs, const double *ms, int64_t ntgt, const double *xt,
                  double G, double *phi, double *acc) {
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < ntgt; ++t) {
    double p = 0, a[3] = {0, 0, 0};
    for (int64_t i = 0; i < nsrc; ++i) {
      double R[3] = {xt[3 * t] - xs[3 * i], xt[3 * t + 1] - xs[3 * i + 1], xt[3 * t + 2] - xs[3 * i + 2]};
      if (R[0] == 0.0 && R[1] == 0.0 && R[2] == 0.0) continue;
      op_p2p(R, ms[i], &p, a);
    }
    phi[t] = G * p;
    for (int k = 0; k < 3; ++k) acc[3 * t + k] = G * a[k];
  }
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* periodic boxes: Ewald sums                                          */
/* ------------------------------------------------------------------ */
/*
 * Potential of unit masses on the lattice x + n L (all integer n) with a
 * uniform neutralising background, zero on average over the box (Ewald):
 *   Psi(r) = sum_n erfc(al |r + nL|)/|r + nL|
 *          + 4 pi / L^3 sum_{k != 0} exp(-k^2 / (4 al^2)) / k^2 cos(k.r) - pi / (al^2 L^3),
 * k = 2 pi m / L.  The split parameter al changes nothing in exact arithmetic.
 *
 * Cartesian derivatives of a radial function h(|x|) follow from its iterated
 * radial derivatives h_m = ((1/rho) d/drho)^m h: with R_0^(m) = h_m,
 * R_{g+e_i}^(m) = x_i R_g^(m+1) + g_i R_{g-e_i}^(m+1), and d^g h = R_g^(0).
 */
#define OR_PI 3.14159265358979323846
/* ranges for 2 <= al L <= 3: every term left out is below 1e-18 of the kept ones */
#define EW_NREAL 4   /* lattice tensors (derivatives to order 10): images |n_i| <= 4 */
#define EW_NRECIP 10 /*   and reciprocal vectors |m_i| <= 10 */
#define EW_NREAL_D 3 /* direct sums (potential and force): images |n_i| <= 3 */
#define EW_NRECIP_D 6 /*   and reciprocal vectors |m_i| <= 6 */

/* h_m of h = erfc(al rho)/rho (sg = +1) or erf(al rho)/rho (sg = -1), rho > 0, m <= n */
static void radial_erfc(int n, double rho, double al, int sg, double *hm) {
  double r2 = rho * rho;
  double B = erfc(al * rho) / rho, inv = 1.0 / rho, odd = 1.0;   /* odd = (2m-1)!! */
  double t = exp(-al * al * r2) * 2.0 * al / sqrt(OR_PI);         /* (2 al^2)^(m-1) 2 al/sqrt(pi) e^{-al^2 rho^2} */
  for (int m = 0; m <= n; ++m) {
    /* ((1/rho) d/drho)^m erfc(al rho)/rho = (-1)^m B_m,
       B_m = ((2m - 1) B_{m-1} + (2 al^2)^(m-1) 2 al/sqrt(pi) e^{-al^2 rho^2}) / rho^2 */
    if (m > 0) {
      B = ((2.0 * m - 1.0) * B + t) / r2;
      t *= 2.0 * al * al;
      odd *= (2.0 * m - 1.0);
      inv /= r2;
    }
    const double sgm = (m & 1) ? -1.0 : 1.0;
    hm[m] = sg > 0 ? sgm * B : sgm * (odd * inv - B);   /* erf = 1 - erfc; (1/rho)' chain gives (2m-1)!!/rho^(2m+1) */
  }
}

/* all d^g h at x for |g| <= n from hm[0..n] */
static void radial_tensor(int n, const double x[3], const double *hm, double *out) {
  int K = nmi_of(n);
  double *R = (double *)malloc(sizeof(double) * (size_t)(n + 1) * K);
#define RR(m, g) R[(size_t)(m) * K + (g)]
  for (int g = 0; g < K; ++g) {
    const int *gg = g_mi[g];
    int d = gg[0] + gg[1] + gg[2];
    for (int m = 0; m + d <= n; ++m) {
      if (d == 0) { RR(m, g) = hm[m]; continue; }
      int i = gg[0] > 0 ? 0 : (gg[1] > 0 ? 1 : 2);
      int q[3] = {gg[0], gg[1], gg[2]};
      q[i] -= 1;                               /* g = q + e_i */
      double v = x[i] * RR(m + 1, g_idx[q[0]][q[1]][q[2]]);
      if (q[i] > 0) {
        int w[3] = {q[0], q[1], q[2]};
        w[i] -= 1;
        v += q[i] * RR(m + 1, g_idx[w[0]][w[1]][w[2]]);
      }
      RR(m, g) = v;
    }
  }
  for (int g = 0; g < K; ++g) out[g] = RR(0, g);
#undef RR
  free(R);
}

/* d^g of Psi(r) - sum over the 27 images n in {-1,0,1}^3 of 1/|r + nL| at r = d
   (|d_i| < L), |g| <= n, negated: D^lat_g(d) in the convention D_g = d^g(-1/r). */
int oracle_lattice_at(int n, double L, double al, const double d[3], double *out) {
  init_tables();
  if (n < 0 || n > PMAX || !(L > 0) || !(al > 0)) return OR_E_INVALID;
  for (int k = 0; k < 3; ++k)
    if (!(fabs(d[k]) < L)) return OR_E_INVALID;
  int K = nmi_of(n);
  double *acc = (double *)calloc(K, sizeof(double)), *t = (double *)malloc(sizeof(double) * K);
  double hm[PMAX + 2];
  for (int a = -EW_NREAL; a <= EW_NREAL; ++a)
    for (int b = -EW_NREAL; b <= EW_NREAL; ++b)
      for (int c = -EW_NREAL; c <= EW_NREAL; ++c) {
        int near = abs(a) <= 1 && abs(b) <= 1 && abs(c) <= 1;
        double x[3] = {d[0] + a * L, d[1] + b * L, d[2] + c * L};
        double rho = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        if (rho == 0.0) {
          /* -erf(al rho)/rho at rho -> 0: h_m(0) = 2 al/sqrt(pi) (-1)^m (2 al^2)^m / (2m + 1) */
          for (int m = 0; m <= n; ++m)
            hm[m] = -2.0 * al / sqrt(OR_PI) * ((m & 1) ? -1.0 : 1.0) * pow(2.0 * al * al, m) / (2.0 * m + 1.0);
        } else {
          radial_erfc(n, rho, al, near ? -1 : +1, hm);
          if (near)
            for (int m = 0; m <= n; ++m) hm[m] = -hm[m];
        }
        radial_tensor(n, x, hm, t);
        for (int g = 0; g < K; ++g) acc[g] += t[g];
      }
  /* reciprocal space: d^g cos(k.r) at r = d is Re(i^|g| k^g e^{i k.d}) */
  const double pref = 4.0 * OR_PI / (L * L * L);
  for (int a = -EW_NRECIP; a <= EW_NRECIP; ++a)
    for (int b = -EW_NRECIP; b <= EW_NRECIP; ++b)
      for (int c = -EW_NRECIP; c <= EW_NRECIP; ++c) {
        if (a == 0 && b == 0 && c == 0) continue;
        double k[3] = {2.0 * OR_PI * a / L, 2.0 * OR_PI * b / L, 2.0 * OR_PI * c / L};
        double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        double w = pref * exp(-k2 / (4.0 * al * al)) / k2, kd = k[0] * d[0] + k[1] * d[1] + k[2] * d[2];
        double cs = cos(kd), sn = sin(kd);
        for (int g = 0; g < K; ++g) {
          int dg = g_mi[g][0] + g_mi[g][1] + g_mi[g][2];
          double ph = (dg & 3) == 0 ? cs : (dg & 3) == 1 ? -sn : (dg & 3) == 2 ? -cs : sn;
          acc[g] += w * ph * mono(g_mi[g], k);
        }
      }
  acc[0] -= OR_PI / (al * al * L * L * L);
  for (int g = 0; g < K; ++g) out[g] = -acc[g];
  free(acc); free(t);
  return OR_OK;
}

int oracle_lattice(int n, double L, double al, double *out) {
  const double zero[3] = {0.0, 0.0, 0.0};
  return oracle_lattice_at(n, L, al, zero, out);
}

/* Periodic direct sum: phi = -G sum_j m_j Psi(x_t - x_j) (a source at the target's
   own position contributes its images and the background: Psi minus 1/r at 0),
   a = -grad phi. */
int oracle_direct_periodic(int64_t nsrc, const double *xs, const double *ms, int64_t ntgt, const double *xt,
                           double G, double L, double al, double *phi, double *acc) {
  init_tables();
  if (!(L > 0) || !(al > 0)) return OR_E_INVALID;
  const double pref = 4.0 * OR_PI / (L * L * L);
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < ntgt; ++t) {
    double ps = 0, a[3] = {0, 0, 0};   /* Psi and grad Psi summed over sources, times m */
    for (int64_t i = 0; i < nsrc; ++i) {
      double r[3] = {xt[3 * t] - xs[3 * i], xt[3 * t + 1] - xs[3 * i + 1], xt[3 * t + 2] - xs[3 * i + 2]};
      double m = ms[i], pv = 0, gv[3] = {0, 0, 0};
      for (int na = -EW_NREAL_D; na <= EW_NREAL_D; ++na)
        for (int nb = -EW_NREAL_D; nb <= EW_NREAL_D; ++nb)
          for (int nc = -EW_NREAL_D; nc <= EW_NREAL_D; ++nc) {
            double x[3] = {r[0] + na * L, r[1] + nb * L, r[2] + nc * L};
            double rho2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
            if (rho2 == 0.0) {
              pv -= 2.0 * al / sqrt(OR_PI);   /* erfc(al rho)/rho - 1/rho at rho -> 0 */
              continue;
            }
            double rho = sqrt(rho2), ec = erfc(al * rho) / rho;
            pv += ec;
            /* d/drho (erfc(al rho)/rho) / rho */
            double d1 = -(ec + 2.0 * al / sqrt(OR_PI) * exp(-al * al * rho2)) / rho2;
            for (int k = 0; k < 3; ++k) gv[k] += d1 * x[k];
          }
      for (int ma = -EW_NRECIP_D; ma <= EW_NRECIP_D; ++ma)
        for (int mb = -EW_NRECIP_D; mb <= EW_NRECIP_D; ++mb)
          for (int mc = -EW_NRECIP_D; mc <= EW_NRECIP_D; ++mc) {
            if (ma == 0 && mb == 0 && mc == 0) continue;
            double k[3] = {2.0 * OR_PI * ma / L, 2.0 * OR_PI * mb / L, 2.0 * OR_PI * mc / L};
            double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
            double w = pref * exp(-k2 / (4.0 * al * al)) / k2, kr = k[0] * r[0] + k[1] * r[1] + k[2] * r[2];
            pv += w * cos(kr);
            for (int q = 0; q < 3; ++q) gv[q] -= w * sin(kr) * k[q];
          }
      pv -= OR_PI / (al * al * L * L * L);
      ps += m * pv;
      for (int k = 0; k < 3; ++k) a[k] += m * gv[k];
    }
    phi[t] = -G * ps;
    for (int k = 0; k < 3; ++k) acc[3 * t + k] = G * a[k];   /* a = -grad(-G Psi) = G grad Psi */
  }
  return OR_OK;
}

/* Periodic boxes for the FMM: needs levelmin >= 3 (the intermediate field of
   the coarsest leaves then reads level 2), re-checks the grading on the torus
   and fills the level-2 far operators (8 target octants x 7^3 offsets). */
int oracle_set_periodic(oracle_state *s, int on) {
  if (!s) return OR_E_INVALID;
  if (!on) { s->periodic = 0; return OR_OK; }
  if (s->levelmin < 3) return OR_E_UNSUPPORTED;
  s->periodic = 1;
  int rc = check_grading(s);
  if (rc) { s->periodic = 0; return rc; }
  free(s->lat);
  int K = s->K;
  s->lat = (double *)malloc(sizeof(double) * 8 * 343 * (size_t)K);
  double *D = (double *)malloc(sizeof(double) * K), *Dl = (double *)malloc(sizeof(double) * K);
  if (!s->lat || !D || !Dl) { free(D); free(Dl); s->periodic = 0; return OR_E_NOMEM; }
  const double h2 = s->boxlen / 4.0;
  for (int di = 0; di < 343 && rc == OR_OK; ++di) {
    /* source offset in level-2 cells, e = c_s - c_y */
    const int e[3] = {di % 7 - 3, (di / 7) % 7 - 3, di / 49 - 3};
    const double R[3] = {-e[0] * h2, -e[1] * h2, -e[2] * h2};   /* c_y - c_s */
    rc = oracle_lattice_at(s->p, s->boxlen, 1.8 / s->boxlen, R, Dl);
    for (int oy = 0; oy < 8 && rc == OR_OK; ++oy) {
      double *T = &s->lat[((size_t)oy * 343 + di) * K];
      memcpy(T, Dl, sizeof(double) * K);
      /* block images n whose level-1 father image does not touch the target's:
         in level-1 cells that offset is floor((o_y + e + 4 n) / 2) per axis */
      for (int n = 0; n < 27; ++n) {
        const int nn[3] = {n % 3 - 1, (n / 3) % 3 - 1, n / 9 - 1};
        int far = 0;
        for (int k = 0; k < 3; ++k) {
          int v = ((oy >> k) & 1) + e[k] + 4 * nn[k];
          int q = v >= 0 ? v / 2 : -((-v + 1) / 2);
          if (q <= -2 || q >= 2) far = 1;
        }
        if (!far) continue;
        const double Rn[3] = {R[0] - nn[0] * s->boxlen, R[1] - nn[1] * s->boxlen, R[2] - nn[2] * s->boxlen};
        derivs(s->p, Rn, D);
        for (int g = 0; g < K; ++g) T[g] += D[g];
      }
    }
  }
  free(D); free(Dl);
  if (rc) s->periodic = 0;
  return rc;
}

/* ------------------------------------------------------------------ */
/* building blocks exposed for the pins                                */
/* ------------------------------------------------------------------ */
int oracle_nmi(int p) { return nmi_of(p); }
int oracle_multi_index(int p, int32_t *out) {
  init_tables();
  if (p < 0 || p > PMAX) return OR_E_UNSUPPORTED;
  for (int i = 0; i < nmi_of(p); ++i)
    for (int k = 0; k < 3; ++k) out[3 * i + k] = g_mi[i][k];
  return OR_OK;
}
int oracle_derivs(int n, const double *R, double *out) {
  init_tables();
  if (n < 0 || n > PMAX) return OR_E_UNSUPPORTED;
  derivs(n, R, out);
  return OR_OK;
}
/* multipole of point masses about centre c (Eq. eqn:multipole) */
int oracle_multipole(int p, int64_t n, const double *x, const double *m, const double *c, double *M) {
  init_tables();
  int K = nmi_of(p);
  memset(M, 0, sizeof(double) * K);
  for (int64_t i = 0; i < n; ++i) {
    double d[3] = {x[3 * i] - c[0], x[3 * i + 1] - c[1], x[3 * i + 2] - c[2]};
    for (int q = 0; q < K; ++q) M[q] += m[i] * mono(g_mi[q], d);
  }
  return OR_OK;
}
int oracle_m2m(int p, const double *t, const double *M, double *Mout) {
  init_tables();
  memset(Mout, 0, sizeof(double) * nmi_of(p));
  op_m2m(p, t, M, Mout);
  return OR_OK;
}
int oracle_m2l(int p, const double *R, const double *M, double *L) {
  init_tables();
  memset(L, 0, sizeof(double) * nmi_of(p));
  op_m2l(p, p, R, M, L, 1.0);
  return OR_OK;
}
int oracle_l2l(int p, const double *a, const double *L, double *Lout) {
  init_tables();
  memset(Lout, 0, sizeof(double) * nmi_of(p));
  op_l2l(p, a, L, Lout);
  return OR_OK;
}
int oracle_l2p(int p, const double *u, const double *L, double *out4) {
  init_tables();
  double ph = 0, a[3] = {0, 0, 0};
  op_l2p(p, u, L, &ph, a);
  out4[0] = ph; out4[1] = a[0]; out4[2] = a[1]; out4[3] = a[2];
  return OR_OK;
}
int oracle_m2p(int p, const double *R, const double *M, double *out4) {
  init_tables();
  double ph = 0, a[3] = {0, 0, 0};
  op_m2p(p, p, R, M, &ph, a);
  out4[0] = ph; out4[1] = a[0]; out4[2] = a[1]; out4[3] = a[2];
  return OR_OK;
}

/*
 * Literal upward chain for tree j (pin of the definition path): P2M of each
 * level-j leaf into its father oct, then M2M (Eq. eq:M2M_general) level by
 * level.  Writes the FMM cells of T_{j;f} in the same row order as the tree
 * (call after oracle_rebuild); returns the max abs difference relative to the
 * largest monopole.
 */
int oracle_chain_check(oracle_state *s, int j, double *maxrel) {
  if (j <= s->levelmin - 1 || j > s->levelmax || !s->tree[j].built) return OR_E_STATE;
  tree_t *t = &s->tree[j];
  int K = s->K;
  if (j < 2) { *maxrel = 0; return OR_OK; }
  /* bottom FMM level j-1: P2M from leaves */
  grid_t *gb = &t->g[j - 1];
  double *cur = (double *)calloc((size_t)(gb->rows ? gb->rows : 1) * K, sizeof(double));
  int64_t o = s->off[j];
  for (int64_t i = 0; i < s->ncell[j]; ++i) {
    if (s->refined[o + i]) continue;
    const int32_t *c = &s->ijk[3 * (o + i)];
    int64_t c3[3] = {c[0], c[1], c[2]}, f3[3] = {c[0] >> 1, c[1] >> 1, c[2] >> 1};
    int64_t r = hm_get(&gb->map, key3(f3[0], f3[1], f3[2]));
    double x[3], cf[3], d[3];
    centre(s, j, c3, x);
    centre(s, j - 1, f3, cf);
    for (int k = 0; k < 3; ++k) d[k] = x[k] - cf[k];
    for (int q = 0; q < K; ++q) cur[r * K + q] += t->leafmass[i] * mono(g_mi[q], d);
  }
  double worst = 0, scale = 0;
  for (int f = j - 1; f >= 1; --f) {
    grid_t *g = &t->g[f];
    for (int64_t r = 0; r < g->rows; ++r) {
      scale = fmax(scale, fabs(g->coef[r * K]));
      for (int q = 0; q < K; ++q) worst = fmax(worst, fabs(cur[r * K + q] - g->coef[r * K + q]));
    }
    if (f == 1) break;
    grid_t *gp = &t->g[f - 1];
    double *nxt = (double *)calloc((size_t)(gp->rows ? gp->rows : 1) * K, sizeof(double));
    for (int64_t r = 0; r < g->rows; ++r) {
      int64_t c3[3];
      unkey3(g->keys[r], c3);
      int64_t f3[3] = {c3[0] >> 1, c3[1] >> 1, c3[2] >> 1};
      int64_t rp = hm_get(&gp->map, key3(f3[0], f3[1], f3[2]));
      double cc[3], cf[3], tt[3];
      centre(s, f, c3, cc);
      centre(s, f - 1, f3, cf);
      for (int k = 0; k < 3; ++k) tt[k] = cf[k] - cc[k];
      op_m2m(s->p, tt, &cur[r * K], &nxt[rp * K]);
    }
    free(cur);
    cur = nxt;
  }
  free(cur);
  *maxrel = scale > 0 ? worst / scale : worst;
  return OR_OK;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
