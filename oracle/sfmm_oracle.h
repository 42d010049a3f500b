/*
 * sfmm_oracle.h -- serial FP64 CPU oracle for the symmetric fast multipole
 * method (SFMM) gravity solve with adaptive cubic-spline softening.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this code; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load liboracle.so.  It shares no header,
 * table or helper with the HIP path.
 *
 * Everything here is plain, slow and written to be checked against the paper
 * by eye: Bernard, David-Cleris, Price & Lau, "Momentum-conserving
 * self-gravity in the Phantom SPH code" (arXiv 2602.05804).
 *   - softened direct sum ........ Sect. 2, Eq. (softdirectsum)
 *   - mass moments ............... Sect. 2.1, Eq. (massmom)
 *   - M2L (M_k, dM_k) ............ Sect. 2.2, Eq. (dmkdeffmm) and the M_k
 *                                  definition just above it
 *   - MAC + softening criterion .. Sect. 3, the two inequalities on the
 *                                  opening angle and on R_kern*max(h_max)
 *   - per-leaf dual tree walk .... Sect. 3, Algorithms 1 and 2
 *   - L2L (gravity moments) ...... Appendix A.2, Eq. (gravmtranslat)
 *
 * Conventions: positions x are [n][3] row-major FP64; masses m and
 * softening lengths h are [n]; outputs acc [n][3] and pot [n] are in the
 * caller's (original) particle order.  All pointers are host pointers.
 * Functions return 0 on success and a negative value on invalid arguments.
 */
#ifndef SFMM_ORACLE_H
#define SFMM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_PMAX 8 /* highest expansion order the oracle accepts */

/* ---- softening kernel (cubic spline, compact support 2h) --------------- */
double orc_psi_hat(double q);          /* potential shape, psi(r,h) = psi_hat(r/h)/h   */
double orc_f_hat(double q);            /* force shape, f_hat = -d psi_hat / dq        */
double orc_g(double r, double h);      /* f_hat(q)/(h^2 r), finite at r = 0           */
double orc_psi(double r, double h);    /* psi_hat(q)/h                                */

/* ---- multi-index helpers (exported so tests can pin them) -------------- */
int orc_ncoef(int order);              /* number of alpha with |alpha| <= order        */
/* the multi-index of canonical slot k: out[0..2] */
int orc_multi_index(int k, int* out);
/* D_alpha(r) = d^alpha (1/|r|) for all |alpha| <= order, canonical order */
int orc_derivs(int order, const double* r3, double* out);

/* ---- direct softened sum, Eq. (softdirectsum) -------------------------- */
/* include_self adds -G m_i psi(0, h_i) to pot_i (the j = i term). */
int orc_direct(int64_t n, const double* x, const double* m, const double* h,
               double G, int include_self, double* acc, double* pot);
/* the same, for a subset of targets (indices into the caller's order) */
int orc_direct_targets(int64_t n, const double* x, const double* m, const double* h,
                       double G, int include_self, int64_t ntgt, const int64_t* tgt,
                       double* acc, double* pot);

/* ---- tree ------------------------------------------------------------- */
typedef struct orc_tree orc_tree;
orc_tree* orc_tree_build(int64_t n, const double* x, const double* m, const double* h,
                         int leaf_size, int order);
void orc_tree_free(orc_tree* t);
int64_t orc_tree_num_nodes(const orc_tree* t);
int64_t orc_tree_num_leaves(const orc_tree* t);
int orc_tree_max_depth(const orc_tree* t);
int orc_tree_order(const orc_tree* t);
/* sorted position -> caller index; Morton keys in sorted order */
void orc_tree_get_perm(const orc_tree* t, int64_t* perm);
void orc_tree_get_keys(const orc_tree* t, uint64_t* keys);
/* node arrays (length num_nodes); left/right = -1 for leaves; s3 is [nn][3] */
void orc_tree_get_nodes(const orc_tree* t, int64_t* lo, int64_t* hi, int32_t* left,
                        int32_t* right, int32_t* depth, double* s3, double* mass,
                        double* l, double* hmax);
/* mass moments Q~_alpha = sum m b^alpha / alpha!, [nn][orc_ncoef(order)] */
void orc_tree_get_moments(const orc_tree* t, double* Q);
/* node ids of the leaves, in increasing lo (Morton) order */
void orc_tree_get_leaves(const orc_tree* t, int32_t* leaves);

/* ---- Algorithm 1/2 walk of one leaf: its interaction lists ------------- */
/* Writes up to cap entries; returns the number of M2L entries (which may
 * exceed cap) and stores the P2P count in *n_p2p.  m2l_depth[k] is the depth
 * of the target ancestor p_i, m2l_src[k] the source node. */
int64_t orc_leaf_lists(const orc_tree* t, int32_t leaf, double theta, double r_kern,
                       int32_t* m2l_depth, int32_t* m2l_src, int64_t cap_m2l,
                       int32_t* p2p_src, int64_t cap_p2p, int64_t* n_p2p);

/* ---- recursive mutual dual tree traversal: ordered interaction pairs --- */
int64_t orc_mutual_pairs(const orc_tree* t, double theta, double r_kern,
                         int32_t* m2l_tgt, int32_t* m2l_src, int64_t cap_m2l,
                         int32_t* p2p_a, int32_t* p2p_b, int64_t cap_p2p, int64_t* n_p2p);

/* ---- the solve --------------------------------------------------------- */
enum {
  ORC_MODE_PER_LEAF = 0,   /* Algorithm 1/2 with the L2L chain                 */
  ORC_MODE_MUTUAL = 1,     /* recursive mutual DTT + recursive downward pass   */
  ORC_MODE_DIRECT_ANC = 2  /* Algorithm 1/2, each ancestor's expansion
                              evaluated directly at the particle (no L2L)     */
};
typedef struct {
  int64_t n_m2l;           /* M2L evaluations performed (replication included) */
  int64_t n_p2p_pairs;     /* ordered particle pairs evaluated by P2P         */
  int64_t n_leaves_done;   /* leaves whose particles were computed            */
} orc_stats;

/* ntgt < 0: every particle.  Otherwise only the leaves holding the listed
 * caller indices are walked, and acc/pot are [ntgt][3]/[ntgt] in tgt order. */
int orc_solve(const orc_tree* t, double theta, double G, double r_kern, int include_self,
              int mode, int64_t ntgt, const int64_t* tgt, double* acc, double* pot,
              orc_stats* st);

/* Algorithm 1 with the loop over leaves run by OpenMP threads (nthreads <= 0:
 * the OpenMP default); every particle; equal to orc_solve in mode
 * ORC_MODE_PER_LEAF bit for bit.  *threads_used: the threads that ran. */
int orc_solve_parallel(const orc_tree* t, double theta, double G, double r_kern, int include_self,
                       int nthreads, double* acc, double* pot, orc_stats* st, int* threads_used);

/* one-shot convenience: build, solve every particle, free */
int orc_sfmm_solve(int64_t n, const double* x, const double* m, const double* h,
                   double theta, int order, int leaf_size, double G, double r_kern,
                   int include_self, double* acc, double* pot, orc_stats* st);

/* ---- single M2L pair for the truncation tests ---------------------------
 * moments of the source particles about sS, M2L to the target centre sT,
 * L2P at the target particles; no softening (pure 1/r expansion). */
int orc_m2l_pair(int order, int64_t ns, const double* xs, const double* ms, const double* sS,
                 int64_t nt, const double* xt, const double* sT, double G,
                 double* acc, double* pot);

#ifdef __cplusplus
}
#endif
#endif
