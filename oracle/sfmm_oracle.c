/*
 * sfmm_oracle.c -- serial FP64 CPU oracle of the SFMM gravity solve.
 *
 * TEST INFRASTRUCTURE ONLY (see sfmm_oracle.h).  Built with
 * -O2 -ffp-contract=off so that every floating-point operation below is
 * rounded exactly as written.
 *
 * Paper: Bernard et al., arXiv 2602.05804.  Each function names the passage
 * it follows.  Where the paper is silent the reading taken is stated in a
 * comment and listed in the design notes of the repository.
 *
 * Multi-index notation: alpha = (ax, ay, az), |alpha| = ax+ay+az,
 * alpha! = ax! ay! az!, v^alpha = vx^ax vy^ay vz^az.  The paper's symmetric
 * tensor contraction (1/n!) T . b^(n) equals sum_{|alpha|=n} T_alpha b^alpha / alpha!.
 */
#include "sfmm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ======================================================================== */
/* multi-index tables                                                       */
/* ======================================================================== */
#define DMAX (ORC_PMAX + 2) /* derivative orders up to p+1, plus one spare */
#define MAXC (((DMAX + 1) * (DMAX + 2) * (DMAX + 3)) / 6)

static int mi_ready = 0;
static int mi_a[MAXC][3];             /* slot -> alpha                       */
static int mi_idx[DMAX + 1][DMAX + 1][DMAX + 1]; /* alpha -> slot            */
static double fact[DMAX + 1];

/* canonical order: by degree n, then ax descending, then ay descending */
static void mi_init(void) {
  if (mi_ready) return;
  int k = 0;
  for (int n = 0; n <= DMAX; ++n)
    for (int a = n; a >= 0; --a)
      for (int b = n - a; b >= 0; --b) {
        int c = n - a - b;
        mi_a[k][0] = a; mi_a[k][1] = b; mi_a[k][2] = c;
        mi_idx[a][b][c] = k;
        ++k;
      }
  fact[0] = 1.0;
  for (int i = 1; i <= DMAX; ++i) fact[i] = fact[i - 1] * (double)i;
  mi_ready = 1;
}

int orc_ncoef(int order) {
  if (order < 0) return 0;
  return ((order + 1) * (order + 2) * (order + 3)) / 6;
}

int orc_multi_index(int k, int* out) {
  mi_init();
  if (k < 0 || k >= MAXC) return -1;
  out[0] = mi_a[k][0]; out[1] = mi_a[k][1]; out[2] = mi_a[k][2];
  return 0;
}

static int deg(int k) { return mi_a[k][0] + mi_a[k][1] + mi_a[k][2]; }
static double afact(int k) { return fact[mi_a[k][0]] * fact[mi_a[k][1]] * fact[mi_a[k][2]]; }

/* v^alpha / alpha! for every |alpha| <= order */
static void monomials_over_fact(int order, const double* v, double* out) {
  double pw[3][DMAX + 1];
  for (int d = 0; d < 3; ++d) {
    pw[d][0] = 1.0;
    for (int e = 1; e <= order; ++e) pw[d][e] = pw[d][e - 1] * v[d];
  }
  int nc = orc_ncoef(order);
  for (int k = 0; k < nc; ++k)
    out[k] = pw[0][mi_a[k][0]] * pw[1][mi_a[k][1]] * pw[2][mi_a[k][2]] / afact(k);
}

/* ======================================================================== */
/* Green's function derivatives D_alpha(r) = d^alpha (1/|r|)                */
/* Sect. 2.1 names them D_n, the n-th gradient of G(r) = 1/|r|.  They are   */
/* generated from the Taylor coefficients T_alpha = D_alpha / alpha!, which */
/* obey the Laplace-kernel recurrence                                       */
/*   n r^2 T_alpha = -(2n-1) sum_c r_c T_{alpha-e_c} - (n-1) sum_c T_{alpha-2e_c} */
/* with T_0 = 1/|r| (terms with a negative index are absent).               */
/* ======================================================================== */
int orc_derivs(int order, const double* r3, double* out) {
  mi_init();
  if (order < 0 || order > DMAX) return -1;
  double r2 = r3[0] * r3[0] + r3[1] * r3[1] + r3[2] * r3[2];
  if (!(r2 > 0.0)) return -1;
  int nc = orc_ncoef(order);
  double T[MAXC];
  T[0] = 1.0 / sqrt(r2);
  for (int k = 1; k < nc; ++k) {
    const int* a = mi_a[k];
    int n = a[0] + a[1] + a[2];
    double s1 = 0.0, s2 = 0.0;
    for (int c = 0; c < 3; ++c) {
      int b[3] = {a[0], a[1], a[2]};
      if (b[c] >= 1) {
        b[c] -= 1;
        s1 += r3[c] * T[mi_idx[b[0]][b[1]][b[2]]];
        if (b[c] >= 1) {
          b[c] -= 1;
          s2 += T[mi_idx[b[0]][b[1]][b[2]]];
        }
      }
    }
    T[k] = (-(double)(2 * n - 1) * s1 - (double)(n - 1) * s2) / ((double)n * r2);
  }
  for (int k = 0; k < nc; ++k) out[k] = T[k] * afact(k);
  return 0;
}

/* ======================================================================== */
/* softening kernel                                                         */
/* Sect. 2, Eq. (softdirectsum): Phi_i = -G sum_j m_j phi(|x_i-x_j|, eps),  */
/* phi -> 1/r outside the compact support.  The kernel is the M4 cubic      */
/* spline (support 2h), W = w(q)/(pi h^3) with                              */
/*   w = 1 - 3/2 q^2 + 3/4 q^3  (q<1),  w = (2-q)^3/4  (1<=q<2),  0 beyond. */
/* f_hat(q) is the mass enclosed within q (4 pi int_0^q w q'^2 dq'/pi)      */
/* divided by q^2, and psi_hat(q) = int_q^inf f_hat dq', which is 1/q for   */
/* q >= 2.  Both integrals are written out below in closed form.           */
/* ======================================================================== */
double orc_psi_hat(double q) {
  if (q < 1.0) {
    double q2 = q * q;
    return 7.0 / 5.0 - (2.0 / 3.0) * q2 + (3.0 / 10.0) * q2 * q2 - (1.0 / 10.0) * q2 * q2 * q;
  }
  if (q < 2.0) {
    double q2 = q * q;
    return 8.0 / 5.0 - (4.0 / 3.0) * q2 + q2 * q - (3.0 / 10.0) * q2 * q2 +
           (1.0 / 30.0) * q2 * q2 * q - 1.0 / (15.0 * q);
  }
  return 1.0 / q;
}

double orc_f_hat(double q) {
  if (q < 1.0) {
    double q2 = q * q;
    return (4.0 / 3.0) * q - (6.0 / 5.0) * q2 * q + 0.5 * q2 * q2;
  }
  if (q < 2.0) {
    double q2 = q * q;
    return (8.0 / 3.0) * q - 3.0 * q2 + (6.0 / 5.0) * q2 * q - (1.0 / 6.0) * q2 * q2 -
           1.0 / (15.0 * q2);
  }
  return 1.0 / (q * q);
}

/* force per unit separation: f_hat(q) / (h^2 r) = (f_hat(q)/q) / h^3, written
 * in the form that stays finite at r = 0 */
double orc_g(double r, double h) {
  double q = r / h;
  if (q < 1.0) {
    double q2 = q * q;
    return (4.0 / 3.0 - (6.0 / 5.0) * q2 + 0.5 * q2 * q) / (h * h * h);
  }
  if (q < 2.0) {
    double q2 = q * q;
    return (8.0 / 3.0 - 3.0 * q + (6.0 / 5.0) * q2 - (1.0 / 6.0) * q2 * q -
            1.0 / (15.0 * q2 * q)) / (h * h * h);
  }
  return 1.0 / (r * r * r);
}

double orc_psi(double r, double h) { return orc_psi_hat(r / h) / h; }

/* One ordered softened pair (i <- j).  Unequal softening lengths: the two
 * kernels are averaged, which keeps the pair force antisymmetric (the
 * paper does not say how unequal h combine; this is the reading taken). */
static void pair_add(double xi, double yi, double zi, double hi, double xj, double yj,
                     double zj, double mj, double hj, double G, double* a, double* p) {
  double dx = xi - xj, dy = yi - yj, dz = zi - zj;
  double r = sqrt(dx * dx + dy * dy + dz * dz);
  double gs = 0.5 * (orc_g(r, hi) + orc_g(r, hj));
  double ps = 0.5 * (orc_psi(r, hi) + orc_psi(r, hj));
  a[0] -= G * mj * gs * dx;
  a[1] -= G * mj * gs * dy;
  a[2] -= G * mj * gs * dz;
  *p -= G * mj * ps;
}

/* ======================================================================== */
/* direct sum, Sect. 2 Eq. (softdirectsum)                                  */
/* ======================================================================== */
static int check_particles(int64_t n, const double* x, const double* m, const double* h) {
  if (n < 0) return -1;
  if (n > 0 && (!x || !m || !h)) return -1;
  return 0;
}

int orc_direct_targets(int64_t n, const double* x, const double* m, const double* h,
                       double G, int include_self, int64_t ntgt, const int64_t* tgt,
                       double* acc, double* pot) {
  if (check_particles(n, x, m, h)) return -1;
  for (int64_t t = 0; t < ntgt; ++t) {
    int64_t i = tgt ? tgt[t] : t;
    if (i < 0 || i >= n) return -1;
    double a[3] = {0.0, 0.0, 0.0}, p = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      pair_add(x[3 * i], x[3 * i + 1], x[3 * i + 2], h[i], x[3 * j], x[3 * j + 1],
               x[3 * j + 2], m[j], h[j], G, a, &p);
    }
    if (include_self) p -= G * m[i] * orc_psi(0.0, h[i]);
    acc[3 * t] = a[0]; acc[3 * t + 1] = a[1]; acc[3 * t + 2] = a[2];
    pot[t] = p;
  }
  return 0;
}

int orc_direct(int64_t n, const double* x, const double* m, const double* h, double G,
               int include_self, double* acc, double* pot) {
  return orc_direct_targets(n, x, m, h, G, include_self, n, NULL, acc, pot);
}

/* ======================================================================== */
/* tree                                                                     */
/* The paper builds a kd-tree around the centre of mass (Sect. 3); this     */
/* oracle uses the Morton binary radix tree instead (the tree type is free; */
/* parity is defined for this tree):                                        */
/*  - cubic bounding box, 21-bit cells per axis, keys interleaved x>y>z;   */
/*  - particles sorted by (key, caller index);                              */
/*  - a range [lo,hi) with at most leaf_size particles is a leaf; otherwise */
/*    it splits where the highest bit differing between its first and last  */
/*    key flips; ranges of equal keys split on the highest differing bit of */
/*    the two sorted positions.                                             */
/* ======================================================================== */
struct orc_tree {
  int64_t n;
  int leaf_size, order, nc;
  double *xs, *ys, *zs, *ms, *hs; /* particles in sorted order */
  int64_t* perm;                  /* sorted position -> caller index */
  uint64_t* keys;
  int64_t nn, cap;
  int64_t *lo, *hi;
  int32_t *left, *right, *depth, *parent;
  double *s, *mass, *l, *hmax, *Q;
  int32_t* leaves;
  int64_t nleaves;
  int maxdepth;
};

typedef struct { uint64_t key; int64_t idx; } keyidx;

static int cmp_keyidx(const void* a, const void* b) {
  const keyidx* u = (const keyidx*)a;
  const keyidx* v = (const keyidx*)b;
  if (u->key != v->key) return u->key < v->key ? -1 : 1;
  if (u->idx != v->idx) return u->idx < v->idx ? -1 : 1;
  return 0;
}

static uint64_t interleave3(uint64_t cx, uint64_t cy, uint64_t cz) {
  uint64_t k = 0;
  for (int b = 20; b >= 0; --b)
    k = (k << 3) | (((cx >> b) & 1u) << 2) | (((cy >> b) & 1u) << 1) | ((cz >> b) & 1u);
  return k;
}

static int highest_bit(uint64_t v) { /* v != 0 */
  int b = 63;
  while (!((v >> b) & 1u)) --b;
  return b;
}

static int32_t new_node(orc_tree* t) {
  if (t->nn == t->cap) {
    int64_t c = t->cap ? 2 * t->cap : 64;
    t->lo = realloc(t->lo, c * sizeof(int64_t));
    t->hi = realloc(t->hi, c * sizeof(int64_t));
    t->left = realloc(t->left, c * sizeof(int32_t));
    t->right = realloc(t->right, c * sizeof(int32_t));
    t->depth = realloc(t->depth, c * sizeof(int32_t));
    t->parent = realloc(t->parent, c * sizeof(int32_t));
    t->cap = c;
  }
  return (int32_t)(t->nn++);
}

/* split position of an internal range (see the header comment above) */
static int64_t split_of(const orc_tree* t, int64_t lo, int64_t hi) {
  uint64_t a = t->keys[lo], b = t->keys[hi - 1];
  if (a != b) {
    int bit = highest_bit(a ^ b);
    int64_t m = lo;
    while (!((t->keys[m] >> bit) & 1u)) ++m;
    return m;
  }
  int bit = highest_bit((uint64_t)lo ^ (uint64_t)(hi - 1));
  return (int64_t)((((uint64_t)(hi - 1)) >> bit) << bit);
}

static int32_t build_range(orc_tree* t, int64_t lo, int64_t hi, int32_t parent, int depth) {
  int32_t id = new_node(t);
  t->lo[id] = lo; t->hi[id] = hi; t->parent[id] = parent; t->depth[id] = depth;
  t->left[id] = -1; t->right[id] = -1;
  if (depth > t->maxdepth) t->maxdepth = depth;
  if (hi - lo > t->leaf_size) {
    int64_t m = split_of(t, lo, hi);
    int32_t L = build_range(t, lo, m, id, depth + 1);
    int32_t R = build_range(t, m, hi, id, depth + 1);
    t->left[id] = L; t->right[id] = R;
  }
  return id;
}

/* Node geometry.  Mass and centre of mass: a leaf sums m_j and m_j x_j in
 * sorted order; an internal node combines its children as
 * (M_L s_L + M_R s_R) / (M_L + M_R).  The node size l (the paper's l_tgt,
 * l_src, Sect. 3) is read as the largest distance from the centre of mass to
 * a particle of the node; h_max is the largest softening length in it. */
static void geometry(orc_tree* t, int32_t id) {
  if (t->left[id] < 0) {
    double M = 0.0, S[3] = {0.0, 0.0, 0.0}, hm = 0.0;
    for (int64_t j = t->lo[id]; j < t->hi[id]; ++j) {
      M += t->ms[j];
      S[0] += t->ms[j] * t->xs[j];
      S[1] += t->ms[j] * t->ys[j];
      S[2] += t->ms[j] * t->zs[j];
      if (t->hs[j] > hm) hm = t->hs[j];
    }
    t->mass[id] = M;
    for (int d = 0; d < 3; ++d) t->s[3 * id + d] = S[d] / M;
    t->hmax[id] = hm;
  } else {
    int32_t L = t->left[id], R = t->right[id];
    geometry(t, L);
    geometry(t, R);
    double M = t->mass[L] + t->mass[R];
    t->mass[id] = M;
    for (int d = 0; d < 3; ++d)
      t->s[3 * id + d] = (t->mass[L] * t->s[3 * L + d] + t->mass[R] * t->s[3 * R + d]) / M;
    t->hmax[id] = t->hmax[L] > t->hmax[R] ? t->hmax[L] : t->hmax[R];
  }
  double d2max = 0.0;
  for (int64_t j = t->lo[id]; j < t->hi[id]; ++j) {
    double dx = t->xs[j] - t->s[3 * id];
    double dy = t->ys[j] - t->s[3 * id + 1];
    double dz = t->zs[j] - t->s[3 * id + 2];
    double d2 = dx * dx + dy * dy + dz * dz;
    if (d2 > d2max) d2max = d2;
  }
  /* sqrt is monotone, so sqrt of the largest square is the largest distance */
  t->l[id] = sqrt(d2max);
}

/* Mass moments about the node centre, Sect. 2.1 Eq. (massmom), summed over
 * the node's particles directly (Q~_alpha = sum_j m_j b_j^alpha / alpha!). */
static void moments(orc_tree* t) {
  int nc = t->nc;
  double mono[MAXC];
  for (int64_t id = 0; id < t->nn; ++id) {
    double* Q = t->Q + id * nc;
    for (int k = 0; k < nc; ++k) Q[k] = 0.0;
    for (int64_t j = t->lo[id]; j < t->hi[id]; ++j) {
      double b[3] = {t->xs[j] - t->s[3 * id], t->ys[j] - t->s[3 * id + 1],
                     t->zs[j] - t->s[3 * id + 2]};
      monomials_over_fact(t->order, b, mono);
      for (int k = 0; k < nc; ++k) Q[k] += t->ms[j] * mono[k];
    }
  }
}

orc_tree* orc_tree_build(int64_t n, const double* x, const double* m, const double* h,
                         int leaf_size, int order) {
  mi_init();
  if (check_particles(n, x, m, h) || n < 1 || leaf_size < 1 || order < 0 || order > ORC_PMAX)
    return NULL;
  orc_tree* t = calloc(1, sizeof(orc_tree));
  t->n = n; t->leaf_size = leaf_size; t->order = order; t->nc = orc_ncoef(order);
  /* cubic bounding box and Morton keys */
  double mn[3], mx[3];
  for (int d = 0; d < 3; ++d) { mn[d] = x[d]; mx[d] = x[d]; }
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) {
      if (x[3 * i + d] < mn[d]) mn[d] = x[3 * i + d];
      if (x[3 * i + d] > mx[d]) mx[d] = x[3 * i + d];
    }
  double ext = 0.0;
  for (int d = 0; d < 3; ++d)
    if (mx[d] - mn[d] > ext) ext = mx[d] - mn[d];
  keyidx* ki = malloc(n * sizeof(keyidx));
  double scale = ext > 0.0 ? 2097152.0 / ext : 0.0;
  for (int64_t i = 0; i < n; ++i) {
    uint64_t c[3] = {0, 0, 0};
    if (ext > 0.0)
      for (int d = 0; d < 3; ++d) {
        double f = floor((x[3 * i + d] - mn[d]) * scale);
        c[d] = f > 2097151.0 ? 2097151u : (uint64_t)f;
      }
    ki[i].key = interleave3(c[0], c[1], c[2]);
    ki[i].idx = i;
  }
  qsort(ki, n, sizeof(keyidx), cmp_keyidx);
  t->perm = malloc(n * sizeof(int64_t));
  t->keys = malloc(n * sizeof(uint64_t));
  t->xs = malloc(n * sizeof(double)); t->ys = malloc(n * sizeof(double));
  t->zs = malloc(n * sizeof(double)); t->ms = malloc(n * sizeof(double));
  t->hs = malloc(n * sizeof(double));
  for (int64_t i = 0; i < n; ++i) {
    int64_t j = ki[i].idx;
    t->perm[i] = j; t->keys[i] = ki[i].key;
    t->xs[i] = x[3 * j]; t->ys[i] = x[3 * j + 1]; t->zs[i] = x[3 * j + 2];
    t->ms[i] = m[j]; t->hs[i] = h[j];
  }
  free(ki);
  build_range(t, 0, n, -1, 0);
  t->s = malloc(3 * t->nn * sizeof(double));
  t->mass = malloc(t->nn * sizeof(double));
  t->l = malloc(t->nn * sizeof(double));
  t->hmax = malloc(t->nn * sizeof(double));
  t->Q = malloc(t->nn * t->nc * sizeof(double));
  geometry(t, 0);
  moments(t);
  /* leaves in increasing lo order: pre-order creation already gives that */
  t->nleaves = 0;
  for (int64_t id = 0; id < t->nn; ++id)
    if (t->left[id] < 0) t->nleaves++;
  t->leaves = malloc(t->nleaves * sizeof(int32_t));
  int64_t k = 0;
  for (int64_t id = 0; id < t->nn; ++id)
    if (t->left[id] < 0) t->leaves[k++] = (int32_t)id;
  return t;
}

void orc_tree_free(orc_tree* t) {
  if (!t) return;
  free(t->xs); free(t->ys); free(t->zs); free(t->ms); free(t->hs);
  free(t->perm); free(t->keys);
  free(t->lo); free(t->hi); free(t->left); free(t->right); free(t->depth); free(t->parent);
  free(t->s); free(t->mass); free(t->l); free(t->hmax); free(t->Q); free(t->leaves);
  free(t);
}

int64_t orc_tree_num_nodes(const orc_tree* t) { return t->nn; }
int64_t orc_tree_num_leaves(const orc_tree* t) { return t->nleaves; }
int orc_tree_max_depth(const orc_tree* t) { return t->maxdepth; }
int orc_tree_order(const orc_tree* t) { return t->order; }
void orc_tree_get_perm(const orc_tree* t, int64_t* perm) {
  memcpy(perm, t->perm, t->n * sizeof(int64_t));
}
void orc_tree_get_keys(const orc_tree* t, uint64_t* keys) {
  memcpy(keys, t->keys, t->n * sizeof(uint64_t));
}
void orc_tree_get_nodes(const orc_tree* t, int64_t* lo, int64_t* hi, int32_t* left,
                        int32_t* right, int32_t* depth, double* s3, double* mass, double* l,
                        double* hmax) {
  int64_t nn = t->nn;
  if (lo) memcpy(lo, t->lo, nn * sizeof(int64_t));
  if (hi) memcpy(hi, t->hi, nn * sizeof(int64_t));
  if (left) memcpy(left, t->left, nn * sizeof(int32_t));
  if (right) memcpy(right, t->right, nn * sizeof(int32_t));
  if (depth) memcpy(depth, t->depth, nn * sizeof(int32_t));
  if (s3) memcpy(s3, t->s, 3 * nn * sizeof(double));
  if (mass) memcpy(mass, t->mass, nn * sizeof(double));
  if (l) memcpy(l, t->l, nn * sizeof(double));
  if (hmax) memcpy(hmax, t->hmax, nn * sizeof(double));
}
void orc_tree_get_moments(const orc_tree* t, double* Q) {
  memcpy(Q, t->Q, t->nn * t->nc * sizeof(double));
}
void orc_tree_get_leaves(const orc_tree* t, int32_t* leaves) {
  memcpy(leaves, t->leaves, t->nleaves * sizeof(int32_t));
}

/* ======================================================================== */
/* acceptance, Sect. 3                                                      */
/* M2L is allowed when the opening angle (l_tgt + l_src)/d is below theta   */
/* AND the nodes are not closer than l_tgt + l_src + R_kern max(h_max)      */
/* (the second inequality is read as an opening condition, so that every   */
/* pair inside a softening kernel is summed particle by particle).  d is   */
/* the distance between the two centres of mass.  Both tests are taken in  */
/* squared form; a tie opens the pair.                                     */
/* ======================================================================== */
static int accept(const orc_tree* t, int32_t A, int32_t B, double theta, double r_kern) {
  double dx = t->s[3 * B] - t->s[3 * A];
  double dy = t->s[3 * B + 1] - t->s[3 * A + 1];
  double dz = t->s[3 * B + 2] - t->s[3 * A + 2];
  double d2 = dx * dx + dy * dy + dz * dz;
  double lsum = t->l[A] + t->l[B];
  double hm = t->hmax[A] > t->hmax[B] ? t->hmax[A] : t->hmax[B];
  double rs = lsum + r_kern * hm;
  return (lsum * lsum < (theta * theta) * d2) && (d2 >= rs * rs);
}

static int is_leaf(const orc_tree* t, int32_t id) { return t->left[id] < 0; }

/* ======================================================================== */
/* expansions                                                               */
/* Local coefficients of a node: H_gamma (1 <= |gamma| <= p+1) and P_beta   */
/* (|beta| <= p), stored in the canonical slots of order p+1 and p.         */
/*   P_beta  = (-1)^|beta| sum_{|alpha| <= p-|beta|} D_{alpha+beta} Q~_alpha */
/*     (the paper's M_k, Sect. 2.2)                                         */
/*   H_gamma = (-1)^{|gamma|+1} sum_{|alpha| <= p+1-|gamma|} D_{alpha+gamma} Q~_alpha */
/*     so that H_{beta+e_c} is the (beta,c) component of dM_k, Eq. (dmkdeffmm) */
/* The potential is Phi = -G sum_beta a^beta/beta! P_beta and the           */
/* acceleration a_c = -G sum_beta a^beta/beta! H_{beta+e_c}.                */
/* ======================================================================== */
typedef struct { int p, nH, nP; } expn;

static expn expn_of(int p) {
  expn e;
  e.p = p; e.nH = orc_ncoef(p + 1); e.nP = orc_ncoef(p);
  return e;
}

/* add M2L(target centre sT <- source with centre sS, moments Q) */
static void m2l_add(expn e, const double* sT, const double* sS, const double* Q, double* H,
                    double* P) {
  double r[3] = {sS[0] - sT[0], sS[1] - sT[1], sS[2] - sT[2]};
  double D[MAXC];
  orc_derivs(e.p + 1, r, D);
  int nq = orc_ncoef(e.p);
  for (int g = 1; g < e.nH; ++g) {
    int ng = deg(g);
    double acc = 0.0;
    for (int a = 0; a < nq; ++a) {
      if (deg(a) > e.p + 1 - ng) continue;
      int ag = mi_idx[mi_a[a][0] + mi_a[g][0]][mi_a[a][1] + mi_a[g][1]][mi_a[a][2] + mi_a[g][2]];
      acc += D[ag] * Q[a];
    }
    H[g] += ((ng + 1) % 2 ? -1.0 : 1.0) * acc;
  }
  for (int b = 0; b < e.nP; ++b) {
    int nb = deg(b);
    double acc = 0.0;
    for (int a = 0; a < nq; ++a) {
      if (deg(a) > e.p - nb) continue;
      int ab = mi_idx[mi_a[a][0] + mi_a[b][0]][mi_a[a][1] + mi_a[b][1]][mi_a[a][2] + mi_a[b][2]];
      acc += D[ab] * Q[a];
    }
    P[b] += (nb % 2 ? -1.0 : 1.0) * acc;
  }
}

/* L2L, Appendix A.2 Eq. (gravmtranslat): re-centre the local coefficients
 * by h = s_new - s_old:  C'_gamma = sum_{eta >= gamma} C_eta h^(eta-gamma)/(eta-gamma)! */
static void l2l(expn e, const double* h, const double* H, const double* P, double* Ho,
                double* Po) {
  double mono[MAXC];
  monomials_over_fact(e.p + 1, h, mono);
  for (int g = 0; g < e.nH; ++g) {
    double acc = 0.0;
    for (int k = 0; k < e.nH; ++k) {
      int d0 = mi_a[k][0] - mi_a[g][0], d1 = mi_a[k][1] - mi_a[g][1], d2 = mi_a[k][2] - mi_a[g][2];
      if (d0 < 0 || d1 < 0 || d2 < 0) continue;
      acc += H[k] * mono[mi_idx[d0][d1][d2]];
    }
    Ho[g] = acc;
  }
  for (int b = 0; b < e.nP; ++b) {
    double acc = 0.0;
    for (int k = 0; k < e.nP; ++k) {
      int d0 = mi_a[k][0] - mi_a[b][0], d1 = mi_a[k][1] - mi_a[b][1], d2 = mi_a[k][2] - mi_a[b][2];
      if (d0 < 0 || d1 < 0 || d2 < 0) continue;
      acc += P[k] * mono[mi_idx[d0][d1][d2]];
    }
    Po[b] = acc;
  }
}

/* L2P: evaluate the local expansion at offset a = x_i - s (Sect. 2.2) */
static void l2p(expn e, const double* a, const double* H, const double* P, double G,
                double* acc, double* pot) {
  double mono[MAXC];
  monomials_over_fact(e.p, a, mono);
  double f[3] = {0.0, 0.0, 0.0}, ph = 0.0;
  for (int b = 0; b < e.nP; ++b) {
    for (int c = 0; c < 3; ++c) {
      int bc[3] = {mi_a[b][0], mi_a[b][1], mi_a[b][2]};
      bc[c] += 1;
      f[c] += H[mi_idx[bc[0]][bc[1]][bc[2]]] * mono[b];
    }
    ph += P[b] * mono[b];
  }
  for (int c = 0; c < 3; ++c) acc[c] -= G * f[c];
  *pot -= G * ph;
}

/* ======================================================================== */
/* Algorithm 1/2: the walk of one leaf                                      */
/* ======================================================================== */
typedef struct { int32_t k, src; } pair_t;
typedef struct { pair_t* v; int64_t n, cap; } stack_t_;
static void push(stack_t_* s, int32_t k, int32_t src) {
  if (s->n == s->cap) {
    s->cap = s->cap ? 2 * s->cap : 64;
    s->v = realloc(s->v, s->cap * sizeof(pair_t));
  }
  s->v[s->n].k = k; s->v[s->n].src = src; s->n++;
}

typedef struct { int32_t* v; int64_t n, cap; } ilist;
static void ipush(ilist* l, int32_t x) {
  if (l->n == l->cap) {
    l->cap = l->cap ? 2 * l->cap : 64;
    l->v = realloc(l->v, l->cap * sizeof(int32_t));
  }
  l->v[l->n++] = x;
}

/* the leaf's ancestors p_0 (root) ... p_d (the leaf); returns d + 1 */
static int leaf_branch(const orc_tree* t, int32_t leaf, int32_t* br) {
  int d = t->depth[leaf];
  int32_t id = leaf;
  for (int k = d; k >= 0; --k) { br[k] = id; id = t->parent[id]; }
  return d + 1;
}

/* Sect. 3: the interaction set of a leaf L with ancestors p_0 .. p_d is found
 * by testing pairs (p_k, S) of an ancestor and a source node, starting from
 * (p_0, root).  Each tested pair is classified:
 *   M2L    S is not p_k and the pair passes both criteria (opening angle and
 *          softening): S's moments act on p_k's field moments;
 *   OPEN   otherwise.
 * An opened pair is resolved by the pairs it leads to:
 *   S a leaf, p_k = L         -> P2P: L's particles meet S's directly;
 *   S a leaf, p_k above L     -> (p_{k+1}, S): the same source meets the next
 *                                ancestor on L's branch;
 *   S internal                -> (p_j, S_left), (p_j, S_right) with j = k + 1,
 *                                or j = k once p_k is L itself (a leaf target
 *                                lowers the source until it meets leaves).
 * The pairs still to be tested are kept last-in first-out (the right child
 * is tested first); the order fixes only the order of each list, not its
 * content.  Callbacks collect the results. */
typedef void (*m2l_cb)(void* ctx, int k, int32_t src);
typedef void (*p2p_cb)(void* ctx, int32_t src);

enum { PAIR_M2L = 0, PAIR_OPEN = 1 };
static int classify_pair(const orc_tree* t, int32_t tgt, int32_t src, double theta,
                         double r_kern) {
  if (tgt != src && accept(t, tgt, src, theta, r_kern)) return PAIR_M2L;
  return PAIR_OPEN;
}

static void walk_leaf(const orc_tree* t, const int32_t* br, int d, double theta, double r_kern,
                      m2l_cb on_m2l, p2p_cb on_p2p, void* ctx) {
  stack_t_ todo = {0};
  push(&todo, 0, 0);
  while (todo.n > 0) {
    const pair_t e = todo.v[--todo.n];
    if (classify_pair(t, br[e.k], e.src, theta, r_kern) == PAIR_M2L) {
      on_m2l(ctx, e.k, e.src);
      continue;
    }
    const int at_leaf = e.k == d;
    if (is_leaf(t, e.src)) {
      if (at_leaf) on_p2p(ctx, e.src);
      else push(&todo, e.k + 1, e.src);
    } else {
      const int j = at_leaf ? e.k : e.k + 1;
      push(&todo, j, t->left[e.src]);
      push(&todo, j, t->right[e.src]);
    }
  }
  free(todo.v);
}

typedef struct {
  int32_t *dep, *src, *p2p;
  int64_t cap, cap2, n, n2;
} lists_ctx;
static void lists_m2l(void* c, int k, int32_t s) {
  lists_ctx* x = (lists_ctx*)c;
  if (x->n < x->cap) { x->dep[x->n] = k; x->src[x->n] = s; }
  x->n++;
}
static void lists_p2p(void* c, int32_t s) {
  lists_ctx* x = (lists_ctx*)c;
  if (x->n2 < x->cap2) x->p2p[x->n2] = s;
  x->n2++;
}

int64_t orc_leaf_lists(const orc_tree* t, int32_t leaf, double theta, double r_kern,
                       int32_t* m2l_depth, int32_t* m2l_src, int64_t cap_m2l, int32_t* p2p_src,
                       int64_t cap_p2p, int64_t* n_p2p) {
  if (leaf < 0 || leaf >= t->nn || !is_leaf(t, leaf)) return -1;
  int32_t br[256];
  if (t->depth[leaf] >= 256) return -1;
  int d = leaf_branch(t, leaf, br) - 1;
  lists_ctx c = {m2l_depth, m2l_src, p2p_src, cap_m2l, cap_p2p, 0, 0};
  walk_leaf(t, br, d, theta, r_kern, lists_m2l, lists_p2p, &c);
  if (n_p2p) *n_p2p = c.n2;
  return c.n;
}

/* per-leaf solve context: the parent buffers dM_{p_k} and the neighbour cache */
typedef struct {
  const orc_tree* t;
  expn e;
  const int32_t* br;
  double* dM; /* (d+1) x (nH + nP) */
  ilist nb;
  int64_t n_m2l;
} solve_ctx;
static void solve_m2l(void* c, int k, int32_t s) {
  solve_ctx* x = (solve_ctx*)c;
  const orc_tree* t = x->t;
  double* H = x->dM + (int64_t)k * (x->e.nH + x->e.nP);
  m2l_add(x->e, t->s + 3 * x->br[k], t->s + 3 * s, t->Q + (int64_t)s * t->nc, H, H + x->e.nH);
  x->n_m2l++;
}
static void solve_p2p(void* c, int32_t s) { ipush(&((solve_ctx*)c)->nb, s); }

static int solve_leaf(const orc_tree* t, int32_t leaf, double theta, double G, double r_kern,
                      int include_self, int mode, double* acc_s, double* pot_s, orc_stats* st) {
  expn e = expn_of(t->order);
  int32_t br[256];
  if (t->depth[leaf] >= 256) return -1;
  int d = leaf_branch(t, leaf, br) - 1;
  int nHP = e.nH + e.nP;
  solve_ctx c;
  c.t = t; c.e = e; c.br = br;
  c.dM = calloc((size_t)(d + 1) * nHP, sizeof(double));
  c.nb.v = NULL; c.nb.n = 0; c.nb.cap = 0; c.n_m2l = 0;
  walk_leaf(t, br, d, theta, r_kern, solve_m2l, solve_p2p, &c);
  /* carry the field moments down the branch (L2L, Eq. gravmtranslat), adding
   * each ancestor's own M2L sum on the way */
  double* loc = malloc(nHP * sizeof(double));
  double* tmp = malloc(nHP * sizeof(double));
  memcpy(loc, c.dM, nHP * sizeof(double));
  for (int k = 1; k <= d; ++k) {
    double hv[3];
    for (int q = 0; q < 3; ++q) hv[q] = t->s[3 * br[k] + q] - t->s[3 * br[k - 1] + q];
    l2l(e, hv, loc, loc + e.nH, tmp, tmp + e.nH);
    for (int q = 0; q < nHP; ++q) loc[q] = tmp[q] + c.dM[(int64_t)k * nHP + q];
  }
  const double* sl = t->s + 3 * leaf;
  for (int64_t i = t->lo[leaf]; i < t->hi[leaf]; ++i) {
    double a[3] = {0.0, 0.0, 0.0}, p = 0.0;
    double xi[3] = {t->xs[i], t->ys[i], t->zs[i]};
    if (mode == ORC_MODE_DIRECT_ANC) {
      for (int k = 0; k <= d; ++k) {
        const double* sk = t->s + 3 * br[k];
        double off[3] = {xi[0] - sk[0], xi[1] - sk[1], xi[2] - sk[2]};
        const double* Hk = c.dM + (int64_t)k * nHP;
        l2p(e, off, Hk, Hk + e.nH, G, a, &p);
      }
    } else {
      double off[3] = {xi[0] - sl[0], xi[1] - sl[1], xi[2] - sl[2]};
      l2p(e, off, loc, loc + e.nH, G, a, &p);
    }
    for (int64_t q = 0; q < c.nb.n; ++q) {
      int32_t s = c.nb.v[q];
      for (int64_t j = t->lo[s]; j < t->hi[s]; ++j) {
        if (j == i) continue;
        pair_add(xi[0], xi[1], xi[2], t->hs[i], t->xs[j], t->ys[j], t->zs[j], t->ms[j],
                 t->hs[j], G, a, &p);
        if (st) st->n_p2p_pairs++;
      }
    }
    if (include_self) p -= G * t->ms[i] * orc_psi(0.0, t->hs[i]);
    acc_s[3 * i] = a[0]; acc_s[3 * i + 1] = a[1]; acc_s[3 * i + 2] = a[2];
    pot_s[i] = p;
  }
  if (st) { st->n_m2l += c.n_m2l; st->n_leaves_done++; }
  free(c.dM); free(c.nb.v); free(loc); free(tmp);
  return 0;
}

/* ======================================================================== */
/* recursive mutual dual tree traversal (the serial walk the paper starts  */
/* from, Sect. 3): interact(A, B) over ordered node pairs from (root,root), */
/* M2L into each target's local buffer, then a recursive downward pass.    */
/* ======================================================================== */
typedef struct {
  const orc_tree* t;
  expn e;
  double theta, r_kern, G;
  double* loc; /* nn x (nH+nP) */
  double *acc_s, *pot_s;
  int32_t *mt, *ms_, *pa, *pb;
  int64_t cap, cap2, n, n2;
  int64_t pairs;
} mutual_ctx;

static void mutual_p2p(mutual_ctx* c, int32_t A, int32_t B) {
  const orc_tree* t = c->t;
  if (c->pa) {
    if (c->n2 < c->cap2) { c->pa[c->n2] = A; c->pb[c->n2] = B; }
    c->n2++;
  }
  if (!c->acc_s) return;
  for (int64_t i = t->lo[A]; i < t->hi[A]; ++i)
    for (int64_t j = t->lo[B]; j < t->hi[B]; ++j) {
      if (i == j) continue;
      pair_add(t->xs[i], t->ys[i], t->zs[i], t->hs[i], t->xs[j], t->ys[j], t->zs[j], t->ms[j],
               t->hs[j], c->G, c->acc_s + 3 * i, c->pot_s + i);
      c->pairs++;
    }
}

static void interact(mutual_ctx* c, int32_t A, int32_t B) {
  const orc_tree* t = c->t;
  if (A == B) {
    if (is_leaf(t, A)) { mutual_p2p(c, A, A); return; }
    int32_t ch[2] = {t->left[A], t->right[A]};
    for (int u = 0; u < 2; ++u)
      for (int v = 0; v < 2; ++v) interact(c, ch[u], ch[v]);
    return;
  }
  if (accept(t, A, B, c->theta, c->r_kern)) {
    if (c->mt) {
      if (c->n < c->cap) { c->mt[c->n] = A; c->ms_[c->n] = B; }
      c->n++;
    }
    if (c->loc) {
      double* H = c->loc + (int64_t)A * (c->e.nH + c->e.nP);
      m2l_add(c->e, t->s + 3 * A, t->s + 3 * B, t->Q + (int64_t)B * t->nc, H, H + c->e.nH);
    }
    return;
  }
  int la = is_leaf(t, A), lb = is_leaf(t, B);
  if (la && lb) { mutual_p2p(c, A, B); return; }
  if (lb) { interact(c, t->left[A], B); interact(c, t->right[A], B); return; }
  if (la) { interact(c, A, t->left[B]); interact(c, A, t->right[B]); return; }
  int32_t ca[2] = {t->left[A], t->right[A]}, cb[2] = {t->left[B], t->right[B]};
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) interact(c, ca[u], cb[v]);
}

static void downward(mutual_ctx* c, int32_t id) {
  const orc_tree* t = c->t;
  int nHP = c->e.nH + c->e.nP;
  double* L = c->loc + (int64_t)id * nHP;
  if (is_leaf(t, id)) {
    for (int64_t i = t->lo[id]; i < t->hi[id]; ++i) {
      double off[3] = {t->xs[i] - t->s[3 * id], t->ys[i] - t->s[3 * id + 1],
                       t->zs[i] - t->s[3 * id + 2]};
      l2p(c->e, off, L, L + c->e.nH, c->G, c->acc_s + 3 * i, c->pot_s + i);
    }
    return;
  }
  double* tmp = malloc(nHP * sizeof(double));
  int32_t ch[2] = {t->left[id], t->right[id]};
  for (int u = 0; u < 2; ++u) {
    double hv[3];
    for (int q = 0; q < 3; ++q) hv[q] = t->s[3 * ch[u] + q] - t->s[3 * id + q];
    l2l(c->e, hv, L, L + c->e.nH, tmp, tmp + c->e.nH);
    double* Lc = c->loc + (int64_t)ch[u] * nHP;
    for (int q = 0; q < nHP; ++q) Lc[q] += tmp[q];
    downward(c, ch[u]);
  }
  free(tmp);
}

int64_t orc_mutual_pairs(const orc_tree* t, double theta, double r_kern, int32_t* m2l_tgt,
                         int32_t* m2l_src, int64_t cap_m2l, int32_t* p2p_a, int32_t* p2p_b,
                         int64_t cap_p2p, int64_t* n_p2p) {
  mutual_ctx c;
  memset(&c, 0, sizeof(c));
  c.t = t; c.e = expn_of(t->order); c.theta = theta; c.r_kern = r_kern;
  c.mt = m2l_tgt; c.ms_ = m2l_src; c.cap = cap_m2l;
  c.pa = p2p_a; c.pb = p2p_b; c.cap2 = cap_p2p;
  /* NULL output arrays still count */
  int32_t dummy_a, dummy_b;
  if (!c.mt) { c.mt = &dummy_a; c.ms_ = &dummy_b; c.cap = 0; }
  if (!c.pa) { c.pa = &dummy_a; c.pb = &dummy_b; c.cap2 = 0; }
  interact(&c, 0, 0);
  if (n_p2p) *n_p2p = c.n2;
  return c.n;
}

/* ======================================================================== */
/* the solve                                                                */
/* ======================================================================== */
int orc_solve(const orc_tree* t, double theta, double G, double r_kern, int include_self,
              int mode, int64_t ntgt, const int64_t* tgt, double* acc, double* pot,
              orc_stats* st) {
  if (!t || !(theta > 0.0) || !(r_kern >= 0.0)) return -1;
  if (mode < 0 || mode > 2) return -1;
  if (st) memset(st, 0, sizeof(*st));
  int64_t n = t->n;
  double* acc_s = calloc(3 * n, sizeof(double));
  double* pot_s = calloc(n, sizeof(double));
  int rc = 0;
  if (mode == ORC_MODE_MUTUAL) {
    mutual_ctx c;
    memset(&c, 0, sizeof(c));
    c.t = t; c.e = expn_of(t->order); c.theta = theta; c.r_kern = r_kern; c.G = G;
    c.loc = calloc((size_t)t->nn * (c.e.nH + c.e.nP), sizeof(double));
    c.acc_s = acc_s; c.pot_s = pot_s;
    interact(&c, 0, 0);
    downward(&c, 0);
    if (include_self)
      for (int64_t i = 0; i < n; ++i) pot_s[i] -= G * t->ms[i] * orc_psi(0.0, t->hs[i]);
    if (st) { st->n_p2p_pairs = c.pairs; st->n_leaves_done = t->nleaves; }
    free(c.loc);
  } else if (ntgt < 0) {
    for (int64_t q = 0; q < t->nleaves && !rc; ++q)
      rc = solve_leaf(t, t->leaves[q], theta, G, r_kern, include_self, mode, acc_s, pot_s, st);
  } else {
    /* sorted position of each target, then each distinct leaf once */
    int64_t* inv = malloc(n * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) inv[t->perm[i]] = i;
    char* done = calloc(t->nn, 1);
    for (int64_t q = 0; q < ntgt && !rc; ++q) {
      if (tgt[q] < 0 || tgt[q] >= n) { rc = -1; break; }
      int64_t sp = inv[tgt[q]];
      int32_t id = 0;
      while (!is_leaf(t, id)) id = sp < t->lo[t->right[id]] ? t->left[id] : t->right[id];
      if (!done[id]) {
        done[id] = 1;
        rc = solve_leaf(t, id, theta, G, r_kern, include_self, mode, acc_s, pot_s, st);
      }
      acc[3 * q] = acc_s[3 * sp]; acc[3 * q + 1] = acc_s[3 * sp + 1];
      acc[3 * q + 2] = acc_s[3 * sp + 2]; pot[q] = pot_s[sp];
    }
    free(inv); free(done);
    free(acc_s); free(pot_s);
    return rc;
  }
  for (int64_t i = 0; i < n && !rc; ++i) {
    int64_t j = t->perm[i];
    acc[3 * j] = acc_s[3 * i]; acc[3 * j + 1] = acc_s[3 * i + 1];
    acc[3 * j + 2] = acc_s[3 * i + 2]; pot[j] = pot_s[i];
  }
  free(acc_s); free(pot_s);
  return rc;
}

/* Algorithm 1 with its loop over leaves shared among OpenMP threads (the
 * paper parallelises the per-leaf walk over the threads of one node, Sect. 3).
 * Every leaf reads the tree and writes only its own particles' sums, in the
 * same order as the serial loop, so the result equals orc_solve's (mode
 * ORC_MODE_PER_LEAF, every particle) bit for bit.  nthreads <= 0: the OpenMP
 * default.  *threads_used receives the number of threads that ran. */
int orc_solve_parallel(const orc_tree* t, double theta, double G, double r_kern, int include_self,
                       int nthreads, double* acc, double* pot, orc_stats* st, int* threads_used) {
  if (!t || !(theta > 0.0) || !(r_kern >= 0.0)) return -1;
  if (st) memset(st, 0, sizeof(*st));
  int64_t n = t->n;
  double* acc_s = calloc(3 * n, sizeof(double));
  double* pot_s = calloc(n, sizeof(double));
  int rc = 0, used = 1;
  int64_t m2l = 0, pairs = 0, done = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel reduction(+ : m2l, pairs, done)
  {
#ifdef _OPENMP
#pragma omp single
    used = omp_get_num_threads();
#endif
    orc_stats mine;
    memset(&mine, 0, sizeof(mine));
#pragma omp for schedule(dynamic, 16)
    for (int64_t q = 0; q < t->nleaves; ++q) {
      if (solve_leaf(t, t->leaves[q], theta, G, r_kern, include_self, ORC_MODE_PER_LEAF, acc_s,
                     pot_s, &mine)) {
#pragma omp atomic write
        rc = -1;
      }
    }
    m2l += mine.n_m2l; pairs += mine.n_p2p_pairs; done += mine.n_leaves_done;
  }
  if (st) { st->n_m2l = m2l; st->n_p2p_pairs = pairs; st->n_leaves_done = done; }
  if (threads_used) *threads_used = used;
  for (int64_t i = 0; i < n && !rc; ++i) {
    int64_t j = t->perm[i];
    acc[3 * j] = acc_s[3 * i]; acc[3 * j + 1] = acc_s[3 * i + 1];
    acc[3 * j + 2] = acc_s[3 * i + 2]; pot[j] = pot_s[i];
  }
  free(acc_s); free(pot_s);
  return rc;
}

int orc_sfmm_solve(int64_t n, const double* x, const double* m, const double* h, double theta,
                   int order, int leaf_size, double G, double r_kern, int include_self,
                   double* acc, double* pot, orc_stats* st) {
  if (n == 0) return 0;
  orc_tree* t = orc_tree_build(n, x, m, h, leaf_size, order);
  if (!t) return -1;
  int rc = orc_solve(t, theta, G, r_kern, include_self, ORC_MODE_PER_LEAF, -1, NULL, acc, pot, st);
  orc_tree_free(t);
  return rc;
}

/* ======================================================================== */
/* a single M2L between two particle groups, for the truncation tests       */
/* ======================================================================== */
int orc_m2l_pair(int order, int64_t ns, const double* xs, const double* ms, const double* sS,
                 int64_t nt, const double* xt, const double* sT, double G, double* acc,
                 double* pot) {
  mi_init();
  if (order < 0 || order > ORC_PMAX) return -1;
  expn e = expn_of(order);
  int nq = orc_ncoef(order);
  double Q[MAXC], mono[MAXC];
  for (int k = 0; k < nq; ++k) Q[k] = 0.0;
  for (int64_t j = 0; j < ns; ++j) {
    double b[3] = {xs[3 * j] - sS[0], xs[3 * j + 1] - sS[1], xs[3 * j + 2] - sS[2]};
    monomials_over_fact(order, b, mono);
    for (int k = 0; k < nq; ++k) Q[k] += ms[j] * mono[k];
  }
  double* H = calloc(e.nH + e.nP, sizeof(double));
  m2l_add(e, sT, sS, Q, H, H + e.nH);
  for (int64_t i = 0; i < nt; ++i) {
    double a[3] = {xt[3 * i] - sT[0], xt[3 * i + 1] - sT[1], xt[3 * i + 2] - sT[2]};
    acc[3 * i] = acc[3 * i + 1] = acc[3 * i + 2] = 0.0;
    pot[i] = 0.0;
    l2p(e, a, H, H + e.nH, G, acc + 3 * i, pot + i);
  }
  free(H);
  return 0;
}
