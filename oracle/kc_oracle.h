/*
 * kc_oracle.h -- plain, serial, fp64 CPU oracle for the reduced-space
 * branch-and-bound for K-center clustering (Ren et al., "A Global Optimization
 * Algorithm for K-Center Clustering of One Billion Samples").
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library. It shares no code, header
 * or constant with the device library and must never be called from it.
 *
 * Conventions (all functions):
 *   X        row-major samples, x[s*d + a], float64 (the float32 dataset
 *            promoted exactly), s in [0,n), a in [0,d)
 *   boxes    lo[b*d + a], hi[b*d + a]; a node is K consecutive boxes
 *   nodes    CSR: box_off[m] .. box_off[m+1]-1 are the boxes of node m
 *   refs     CSR per box: ref_off[b] .. ref_off[b+1]-1 index rows of ref[r*d+a]
 *   argmax / argmin ties resolve to the lowest sample index.
 * Summation over attributes runs a = 0..d-1 in fp64 (compiled without FMA
 * contraction).
 */
#ifndef KC_ORACLE_H
#define KC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KCO_MAX_K 64

/* Section 3.1, eq (11) and its closed form: squared distance from x to the
 * nearest point of the box [lo, hi] (per attribute the median of lo, x, hi). */
double kco_point_box_min_dist2(const double *x, const double *lo, const double *hi, int d);

/* Section 4.2.1, eq (13) and its closed form: squared distance from x to the
 * farthest point of the box (per attribute the bound farther from x). */
double kco_point_box_max_dist2(const double *x, const double *lo, const double *hi, int d);

/* Squared Euclidean distance. */
double kco_dist2(const double *x, const double *y, int d);

/* Eqs (8)-(11): per node beta(M) = max_s min_k beta_s^k(M^k) and its argmax. */
void kco_lower_bound(const double *X, int64_t n, int d, int32_t n_nodes,
                     const int32_t *box_off, const double *lo, const double *hi,
                     double *lb, int64_t *argmax);

/* Section 3.2: per box, the sample inside the box closest to the box midpoint
 * (-1 if the box holds no sample). */
void kco_candidates(const double *X, int64_t n, int d, int32_t n_boxes,
                    const double *lo, const double *hi, int64_t *cand);

/* Eq (12) / eq (1): per candidate set, max_s min_k ||x_s - c_k||^2 and argmax.
 * centers[(c*k + j)*d + a]. */
void kco_objective(const double *X, int64_t n, int d, int32_t n_sets, int k,
                   const double *centers, double *obj, int64_t *argmax);

/* Algorithm 3 (cluster assignment) and the per-box aggregates Algorithm 4
 * needs, for one node of k boxes at incumbent alpha.
 *   labels[s]   (nullable) assigned cluster, -1 unassigned, -2 excluded from
 *               every cluster by the center-based test
 *   bb_lo/hi, n_in   bounding box / count of S_+^k = X cap M^k cap balls(refs)
 *   asg_min/max, n_asg   per-cluster min / max / count of assigned samples
 *   asg_far     (nullable) per cluster the assigned sample farthest from the
 *               box midpoint (lowest index among equal distances), -1 if none
 * ref_off has k+1 entries (refs of cluster j are rows ref_off[j]..ref_off[j+1]-1).
 * Returns the number of samples excluded from every cluster. */
int64_t kco_tighten_node(const double *X, int64_t n, int d, int k,
                         const double *lo, const double *hi, double alpha,
                         const int32_t *ref_off, const double *ref,
                         double *bb_lo, double *bb_hi, int64_t *n_in,
                         double *asg_min, double *asg_max, int64_t *n_asg,
                         int64_t *asg_far, int8_t *labels);

/* Algorithm 4 closing step: the tightened box of every cluster from the
 * aggregates of kco_tighten_node (box-based tightening with the assigned
 * samples and the refs, intersected with the bounding box of S_+^k).
 * Returns 1 when the node is infeasible (some S_+^k empty or lo > hi). */
int kco_tightened_box(int d, int k, const double *lo, const double *hi, double alpha,
                      const int32_t *ref_off, const double *ref,
                      const double *bb_lo, const double *bb_hi, const int64_t *n_in,
                      const double *asg_min, const double *asg_max, const int64_t *n_asg,
                      double *lo_out, double *hi_out);

/* Section 4.1.3 symmetry breaking on the first attribute: propagates
 * mu_1^1 <= ... <= mu_1^K into the boxes. Returns 1 if a box became empty. */
int kco_symmetry(int d, int k, double *lo, double *hi);

/* Algorithm 5 / Sections 4.2.1-4.2.2: keep[s] = 0 iff sample s is redundant
 * for lower bounding (alpha_s(M) < beta) and for upper bounding (for every
 * box: outside it, or farther than alpha from one of its refs) in every node. */
void kco_reduce_flags(const double *X, int64_t n, int d, int32_t n_nodes,
                      const int32_t *box_off, const double *lo, const double *hi,
                      const int32_t *ref_off, const double *ref,
                      double beta, double alpha, uint8_t *keep);

/* Algorithm 2, farthest first traversal from sample s0: T[0] = s0, then
 * repeatedly the sample farthest from the chosen set. */
void kco_fft(const double *X, int64_t n, int d, int k, int64_t s0, int64_t *T);

/* Exhaustive search over all k-subsets of the samples (eq (1) by enumeration).
 * Ties keep the lexicographically first subset. */
void kco_brute_force(const double *X, int64_t n, int d, int k, double *best, int64_t *ids);

typedef struct {
  int32_t k;
  int32_t i_sr;          /* sample reduction every i_sr node iterations; 0 = off */
  int32_t use_bt;        /* 1: cluster assignment + ball/box tightening; 0: only
                            the centers-on-samples box */
  int32_t use_seeds;     /* 1: K farthest initial seeds when FFT finds them */
  int32_t max_refs;      /* refs kept per cluster (seeds + assigned samples
                            inherited from ancestors); 0 = seeds only */
  int64_t fft_start;     /* first FFT sample */
  int64_t max_nodes;     /* 0 = unlimited */
  double eps;            /* relative gap tolerance; 0 = exact */
} kco_opts;

typedef struct {
  double obj;            /* best objective found (alpha) */
  double lb;             /* global lower bound at exit (== obj when closed) */
  double fft_obj;        /* objective of the root FFT solution */
  int64_t centers[KCO_MAX_K];  /* incumbent center sample ids (original ids) */
  int64_t nodes;         /* node iterations */
  int64_t n_active;      /* samples left after sample reduction */
  int32_t seeds_found;
  int32_t status;        /* 0 = closed (optimal / gap reached), 1 = node limit */
} kco_result;

/* Algorithm 1: branch and bound to the global optimum. */
int kco_solve(const double *X, int64_t n, int d, const kco_opts *opt, kco_result *res);

#ifdef __cplusplus
}
#endif
#endif
