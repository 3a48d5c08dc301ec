/*
 * kc.h -- C ABI of libkc, the MI355X (gfx950) bound-evaluation library for the
 * reduced-space branch and bound of K-center clustering (Ren et al., "A Global
 * Optimization Algorithm for K-Center Clustering of One Billion Samples").
 *
 * Problem (eq (1)): choose K samples as centers to minimise
 *     max_s min_k ||x_s - mu^k||^2 .
 * A branch-and-bound node is a set of K boxes M^k = [lo^k, hi^k] that hold the
 * centers (Section 3). The calls below evaluate, over all samples, the node
 * lower bound (Section 3.1), the objective of candidate centers (Section 3.2),
 * the cluster-assignment and bounds-tightening aggregates (Section 4.1,
 * Algorithms 3-4) and the sample-reduction masks (Section 4.2, Algorithm 5).
 *
 * Conventions for every call
 * --------------------------
 * Memory   All array arguments are DEVICE pointers (hipMalloc / torch cuda
 *          memory) unless the argument says "host". The caller owns every
 *          input and output buffer; the library owns only the scratch memory
 *          inside the handle (grown on demand, freed by kc_destroy).
 * Layouts  Samples: structure of arrays, x[a*ld + s], float32, 0 <= s < n,
 *          0 <= a < d, ld >= n. Boxes: row-major lo[b*d + a], hi[b*d + a].
 *          Nodes: CSR, boxes box_off[m] .. box_off[m+1]-1 belong to node m.
 *          Refs (samples known to belong to a cluster): CSR per box,
 *          rows ref_off[b] .. ref_off[b+1]-1 of ref[r*d + a].
 * Streams  `stream` is a hipStream_t (NULL = the default stream). Every call
 *          except kc_solve, kc_autotune and kc_fft is stream-ordered and
 *          returns once the work is validated and enqueued; KC_OK means
 *          exactly that.
 * Errors   Argument errors return KC_EINVAL synchronously with a message in
 *          kc_last_error. A launch or runtime failure returns KC_EDEVICE.
 *          No C++ exception crosses this boundary. A handle is used by one
 *          host thread at a time. Malformed CSR offsets (non-monotone or out
 *          of range) give unspecified results but never an out-of-bounds
 *          access: kernels clamp every range to the sizes passed on the host.
 * Indices  argmax / argmin ties resolve to the lowest sample index s.
 * Limits   1 <= d <= 16; 1 <= n < 2^31; boxes per node <= 64; refs per box
 *          <= 64.
 *
 * Floating point: distances are float32. Every result that bounds the
 * optimum carries a rigorous forward-error margin (see kc_rel_margin):
 * lower bounds are rounded down, upper bounds rounded up, and every test is
 * made against a threshold moved by the margin so that it can only err on the
 * safe side. kc_objective(precision = 64) evaluates in float64 to certify an
 * incumbent.
 */
#ifndef KC_H
#define KC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kc_handle kc_handle;

typedef enum {
  KC_OK = 0,
  KC_EINVAL = -1,       /* bad argument (message in kc_last_error)            */
  KC_ENOMEM = -2,       /* device allocation of scratch memory failed         */
  KC_EDEVICE = -3,      /* HIP launch / runtime error                         */
  KC_EUNSUPPORTED = -4  /* valid request the library does not implement       */
} kc_status;

/* Samples in device memory (structure of arrays). Values are finite float32
 * numbers; results for NaN or infinite samples are unspecified. The kernels'
 * results do not depend on the order of the samples (argmax ties go to the
 * lowest position), but they run faster when consecutive samples are close:
 * a wavefront whose samples span a small box settles its box tests at once. */
typedef struct {
  const float *x;  /* [d][ld] */
  int64_t n;       /* number of samples                          */
  int64_t ld;      /* leading dimension (elements), ld >= n      */
  int32_t d;       /* attributes, 1..16                          */
  int32_t reserved;
} kc_points;

/* A batch of nodes, each a set of boxes (CSR). */
typedef struct {
  int32_t n_nodes;         /* host: number of nodes, >= 1                  */
  int32_t n_boxes;         /* host: total boxes = box_off[n_nodes]          */
  int32_t k_max;           /* host: upper bound on boxes per node (1..64)   */
  int32_t reserved;
  const int32_t *box_off;  /* [n_nodes+1], device                          */
  const float *lo;         /* [n_boxes][d], device                         */
  const float *hi;         /* [n_boxes][d], device; lo <= hi per attribute  */
} kc_nodes;

/* Samples known to belong to the cluster of each box (Section 4.1.1: initial
 * seeds and assigned samples). Empty set of refs: pass NULL for the struct. */
typedef struct {
  int32_t n_refs;          /* host: total rows of ref                       */
  int32_t max_per_box;     /* host: upper bound on refs per box (0..64)     */
  const int32_t *ref_off;  /* [n_boxes+1], device                          */
  const float *ref;        /* [n_refs][d], device                          */
} kc_refs;

/* ------------------------------------------------------------- handle ---- */

/* Creates a handle bound to HIP device `device`. tune_cache_path (host
 * string, nullable) names a text file where kc_autotune results persist and
 * from which they are loaded. */
kc_status kc_create(kc_handle **h, int device, const char *tune_cache_path);
void kc_destroy(kc_handle *h);
/* Message for the last non-OK status returned on this handle (host string,
 * owned by the handle, valid until the next call). */
const char *kc_last_error(const kc_handle *h);

/* Relative forward-error bound of one float32 squared distance in d
 * attributes: gamma_{d+3} = (d+3)u / (1 - (d+3)u), u = 2^-24. */
double kc_rel_margin(int d);
/* Absolute term covering underflow: (d+3) * 2^-126. */
double kc_abs_margin(int d);

/* ------------------------------------------------------ bound passes ----- */

/* Section 3.1, eqs (8)-(11): for every node m,
 *     beta(M) = max_s min_{k in m} sum_a (x_{s,a} - mid{lo_a^k, x_{s,a}, hi_a^k})^2
 * lb_raw[m]  float32 value as computed,
 * lb_safe[m] float64, <= the exact value of beta(M) on the float32 data
 *            (lb_raw moved down by the margin; never negative),
 * argmax[m]  lowest sample index attaining lb_raw.
 * cand (nullable, [n_boxes]): Section 3.2 upper-bound candidates, per box the
 * lowest-index sample inside the box closest to the box midpoint (float32
 * midpoint and distance), or -1 when the box holds no sample.
 * A node with no boxes gets lb_raw = +inf. */
kc_status kc_lower_bound(kc_handle *h, const kc_points *pts, const kc_nodes *nodes,
                         float *lb_raw, double *lb_safe, int64_t *argmax, int64_t *cand,
                         void *stream);

/* kc_lower_bound for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results, validation and stream semantics as kc_lower_bound
 * (same kernels and tiles), but the per-split partial results (and, for
 * tiles with wavefront decisions, the per-node and per-box values the
 * workgroups share) live in a static device array of KC_NOALLOC_SCRATCH_BYTES
 * per GPU, whose address the
 * handle takes once per device in kc_create; the call makes no device or host
 * allocation and never synchronises. The caller still owns every input and
 * output buffer. A request whose partial results exceed the array (roughly
 * 8 bytes x (n_nodes + n_boxes with cand) x splits, plus 4 bytes per node
 * and box for shared tile values; at most about 2^19
 * node+box slots in total) fails with KC_EINVAL and a message naming the
 * limit. Every call on one GPU shares that GPU's array: calls that overlap on
 * one GPU (several streams or host threads) race and give unspecified
 * results; calls ordered on one stream are safe. */
#define KC_NOALLOC_SCRATCH_BYTES (4u << 20)
kc_status kc_lower_bound_noalloc(kc_handle *h, const kc_points *pts, const kc_nodes *nodes,
                                 float *lb_raw, double *lb_safe, int64_t *argmax, int64_t *cand,
                                 void *stream);

/* Eq (12): for every candidate set c of k centers (centers[(c*k + j)*d + a]),
 *     obj[c] = max_s min_j ||x_s - center_j||^2 ,  argmax[c] its lowest index.
 * precision 32: float32 evaluation, obj rounded UP by the margin (>= exact).
 * precision 64: float64 evaluation (the certificate of an incumbent). */
kc_status kc_objective(kc_handle *h, const kc_points *pts, int32_t n_sets, int32_t k,
                       const float *centers, int32_t precision, double *obj,
                       int64_t *argmax, void *stream);

/* The float32 objective of eq (12) as an upper-bound screen (Section 3.2:
 * only a candidate set that improves the incumbent matters). Sets whose
 * float32 value v is at most `cut` (host float) get exactly what
 * kc_objective(precision = 32) gives; a set with v > cut may stop early and
 * then reports the float32 value of some sample above cut (obj rounded up by
 * the margin from that value, argmax that sample): a lower bound of its
 * objective, above cut. cut = +inf gives kc_objective's results. floor
 * (device, [n_sets], nullable): a lower bound of each set's exact objective
 * -- for centers inside a node's boxes, the node's lower bound (eqs (8)-(11))
 * -- which lets whole tiles of samples below it be skipped from the start;
 * with a valid floor the results are the same, except that a set whose floor
 * (lowered by the float32 margin) already exceeds cut is not evaluated: it
 * reports that lowered floor, with argmax -1. Same layouts as kc_objective;
 * KC_EINVAL on bad sizes or a NaN cut. */
kc_status kc_objective_screen(kc_handle *h, const kc_points *pts, int32_t n_sets, int32_t k,
                              const float *centers, float cut, const double *floor,
                              double *obj, int64_t *argmax, void *stream);

/* Algorithm 2 (farthest first traversal) from n_trials starts at once: trial t
 * begins at sample starts[t] and adds, k-1 times, the sample farthest (float64
 * squared distance, lowest index on ties) from its centers so far. Every step
 * is one float64 kc_objective launch over all trials.
 * starts (host, [n_trials]) are sample positions in 0..n-1; ids (host, out,
 * [n_trials][k]) receive each trial's centers in order; obj (host, out,
 * nullable, [n_trials]) the float64 objective of eq (12) at those centers.
 * Synchronous on `stream`; KC_EINVAL for k outside 1..64, n_trials outside
 * 1..65535 or a start out of range; KC_ENOMEM if its small device buffers
 * cannot be allocated. */
kc_status kc_fft(kc_handle *h, const kc_points *pts, int32_t k, int32_t n_trials,
                 const int64_t *starts, int64_t *ids, double *obj, void *stream);

/* Algorithms 3-4 for every node at incumbent alpha (host double):
 *   center-based assignment: beta_s^k > alpha for all k != k' => s in k';
 *   sample-based assignment (only if every box of the node has refs): for all
 *     k != k' some ref r of box k has ||x_s - r||^2 > 4 alpha => s in k';
 *   S_+^k = samples inside box k within alpha of every ref of box k.
 * Outputs per box b ([n_boxes][d] / [n_boxes]):
 *   bb_lo, bb_hi, n_in     bounding box and count of S_+^k (+inf/-inf if empty)
 *   asg_min, asg_max, n_asg  min / max / count of samples assigned to b
 * per node: n_excl[m]   samples excluded from every box (the node then lies
 *                       above alpha and may be dropped).
 * asg_far (nullable, [n_boxes]): per box the assigned sample farthest from the
 *   box midpoint (float32 midpoint and distance; lowest index among equal
 *   distances), -1 if none -- a sample known to belong to the box's cluster,
 *   usable as a ref by the node's descendants.
 * labels (nullable, [n], only with n_nodes == 1): assigned box within the
 *   node, -1 unassigned, -2 excluded from every box.
 * Tests use thresholds moved by the margin, so assignments are a subset and
 * S_+^k a superset of their exact counterparts. */
kc_status kc_tighten(kc_handle *h, const kc_points *pts, const kc_nodes *nodes, double alpha,
                     const kc_refs *refs, float *bb_lo, float *bb_hi, uint32_t *n_in,
                     float *asg_min, float *asg_max, uint32_t *n_asg, uint32_t *n_excl,
                     int64_t *asg_far, int8_t *labels, void *stream);

/* Algorithm 5 (Sections 4.2.1-4.2.2) over the open nodes:
 *   LB-redundant in M: min_k max_{mu in M^k} ||x_s - mu||^2 < beta
 *   UB-redundant in M: for every box: x_s outside it, or some ref of the box
 *                      farther than alpha
 * A sample redundant in both senses in every node is deleted; the rest are
 * compacted stably into x_out ([d][ld_out], ld_out >= n) and idx_out
 * (idx_in[s], or s when idx_in is NULL). *n_out (device int64) receives the
 * number kept; keep ([n], nullable) the per-sample flag. x_out / idx_out must
 * not overlap the inputs. */
kc_status kc_reduce(kc_handle *h, const kc_points *in, const uint32_t *idx_in,
                    const kc_nodes *open, const kc_refs *refs, double beta, double alpha,
                    uint8_t *keep, float *x_out, uint32_t *idx_out, int64_t ld_out,
                    int64_t *n_out, void *stream);

/* Synchronous: times the launch variants of kc_lower_bound for this shape
 * (with or without the candidate output) on the given stream, keeps the
 * fastest in the handle's table (and the cache file) and returns its time in
 * milliseconds in *best_ms (host, nullable). */
kc_status kc_autotune(kc_handle *h, const kc_points *pts, const kc_nodes *nodes, int32_t with_cand,
                      double *best_ms, void *stream);

/* Synchronous: times the compiled tiles of kc_tighten for this shape (samples
 * per lane, nodes per workgroup sharing one load of the samples, occupancy),
 * keeps the fastest in the handle's table (and the cache file) under the
 * shape's bucket (attribute count, boxes per node, node and sample count
 * buckets, with or without refs) and returns its time in milliseconds in
 * *best_ms (host, nullable). Every tile gives bit-identical results. Its
 * output buffers are allocated and freed inside the call. */
kc_status kc_autotune_tighten(kc_handle *h, const kc_points *pts, const kc_nodes *nodes,
                              double alpha, const kc_refs *refs, double *best_ms, void *stream);

/* -------------------------------------------- branching network ---------- */
/* A 32-64-64-64-1 ReLU network scoring (cluster, attribute) split candidates.
 * Weights: 10,497 values, layout W1[64][32] b1[64] W2[64][64] b2[64]
 * W3[64][64] b3[64] W4[1][64] b4[1]; bf16 copy (uint16 bit patterns) used by
 * forward/backward, float32 master copy updated by Adam. Features are float32
 * [rows][32], rounded to bf16 on load; accumulation is float32. */
#define KC_MLP_PARAMS 10497
#define KC_MLP_IN 32
#define KC_MLP_HID 64

/* score[rows]; act (nullable, [rows][192]) keeps the three ReLU outputs for
 * the backward pass. */
kc_status kc_mlp_forward(kc_handle *h, const uint16_t *w_bf16, const float *feat, int64_t rows,
                         float *score, float *act, void *stream);
/* dw[KC_MLP_PARAMS] = gradient of sum_r dscore[r] * score[r] (overwritten). */
kc_status kc_mlp_backward(kc_handle *h, const uint16_t *w_bf16, const float *feat,
                          const float *act, const float *dscore, int64_t rows, float *dw,
                          void *stream);
/* Softmax cross-entropy over the rows of each group (grp_off[G+1], target[G]
 * = row index within the group), averaged over groups: loss[0] and
 * dscore[rows]. */
kc_status kc_mlp_loss(kc_handle *h, const float *score, const int32_t *grp_off,
                      const int32_t *target, int32_t n_groups, int64_t rows, float *dscore,
                      float *loss, void *stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on w32, m, v; then
 * w_bf16 = round-to-nearest-even(w32). step >= 1. */
kc_status kc_mlp_adam(kc_handle *h, float *w32, uint16_t *w_bf16, const float *dw, float *m,
                      float *v, int32_t step, float lr, void *stream);

/* ------------------------------------------------- host driver ----------- */

typedef struct {
  int32_t k;            /* clusters, 1..64                                  */
  int32_t batch;        /* nodes popped per pass (>= 1)                     */
  int32_t i_sr;         /* sample reduction every i_sr passes; 0 = off      */
  int32_t use_bt;       /* 1: assignment + tightening (BB+CF+BT)            */
  int32_t use_seeds;    /* 1: K farthest initial seeds when FFT finds them  */
  int32_t max_refs;     /* refs kept per cluster and node: the seeds plus the
                           samples assigned at the node's ancestors (the
                           farthest from its box midpoint per cluster and
                           node); 0 = seeds only                            */
  int32_t branching;    /* 0: max-range rule; 1: learned (needs mlp_w)      */
  int32_t keep_order;   /* 0: after the root pass the active samples are put in
                           Morton order over the root box when n >= 65536 (the
                           certified results do not depend on the order);
                           1: keep the input order                          */
  int32_t node_sr;      /* one-node sample reductions (Section 4.2 with the
                           node's own lower bound): a node bounded over at
                           least node_sr samples may get a sample set of its
                           own, kept by its whole subtree, when that deletes
                           at least a quarter of them. Tries are budgeted by
                           counted work; 65536 suits 10^6..10^9 samples;
                           0 = off                                          */
  int32_t autotune;     /* 1: the first tightening and lower-bound launch of
                           each shape bucket not yet in the handle's table
                           runs the tile sweep (kc_autotune_tighten,
                           kc_autotune) first; later launches and solves on
                           the handle use the table. Results do not depend
                           on the tile                                     */
  int64_t fft_start;    /* first FFT sample                                 */
  int64_t max_nodes;    /* 0 = unlimited                                    */
  double eps_rel;       /* relative gap at which to stop (>= 1e-6 advised)  */
  double time_limit_s;  /* 0 = unlimited                                    */
  const uint16_t *mlp_w;/* device bf16 weights for branching = 1, or NULL   */
  int32_t verbose;      /* 1: progress lines on stderr                      */
  /* Strong-branching labels (training data of the branching network): the
   * first sb_first branched nodes and every sb_every-th after them get every
   * candidate (cluster, attribute) split and bounded; one row per candidate is
   * written to the host arrays below (capacity sb_cap). Candidates, for the
   * labels and for the learned rule, are the sides at least half as wide as
   * the node's widest side. */
  int32_t sb_first;
  int32_t sb_every;     /* 0 = no labels                                    */
  int32_t sb_cap;
  float *sb_feat;       /* host [sb_cap][32] candidate features             */
  float *sb_score;      /* host [sb_cap] product score of the two children:
                           max(dL, e) max(dR, e) / alpha^2, d = child lower
                           bound (alpha for a child with an empty box, at most
                           alpha) minus the node's, e = 1e-6 alpha          */
  int32_t *sb_node;     /* host [sb_cap] ordinal of the labelled node       */
  /* Optional (nullable) host arrays describing each row, so that a score can
   * be recomputed from its definition: the labelled node's tightened boxes
   * (sb_lo, sb_hi: [sb_cap][k*d]), the candidate's (cluster, attribute)
   * (sb_ka: [sb_cap][2]; split as in branching, [lo, m] and [next(m), hi]
   * with m the float32 midpoint rounded down), and the node's lower bound and
   * the incumbent alpha the score was formed with (sb_bounds: [sb_cap][2]). */
  float *sb_lo;
  float *sb_hi;
  int32_t *sb_ka;
  double *sb_bounds;
} kc_opts;

typedef struct {
  double obj;           /* certified incumbent objective (float64 over all samples) */
  double lb;            /* certified global lower bound                      */
  double gap;           /* (obj - lb) / obj                                  */
  double fft_obj;       /* objective of the root FFT centers                 */
  int64_t centers[64];  /* incumbent center sample ids (original indices)    */
  int64_t nodes;        /* nodes processed                                   */
  int64_t passes;       /* kernel passes over the samples                    */
  int64_t evals;        /* sample-box bound evaluations (lower-bound passes) */
  int64_t n_active;     /* samples left after sample reduction               */
  double seconds;       /* wall time                                         */
  double lb_kernel_ms;  /* total time inside kc_lower_bound launches         */
  double tighten_kernel_ms; /* total time inside kc_tighten launches        */
  int64_t tighten_evals;    /* sample-box evaluations of the tightening passes */
  int32_t seeds_found;
  int32_t status;       /* 0 closed (gap <= eps_rel), 1 node limit, 2 time limit,
                           3 no open node left but gap > eps_rel (only when
                           eps_rel is below the float32 margins of the leaves
                           and nodes that closed the search)               */
  int32_t sb_rows;      /* strong-branching rows written                     */
  int32_t sb_nodes;     /* strong-branching nodes labelled                   */
  int64_t node_sr_tries;/* one-node sample reductions run                    */
  int64_t node_sr_kept; /* ... whose sample set a subtree kept               */
  double obj_kernel_ms; /* total time inside the candidates' float32
                           objective launches (kc_objective_screen)          */
  int64_t obj_evals;    /* sample-center evaluations of those launches       */
} kc_result;

/* Algorithm 1 on the device-resident samples `pts` (synchronous; uses its own
 * stream). During the search the best candidate set's rigorous float32 upper
 * bound prunes; its objective is evaluated in float64 over the original
 * samples once, when the search ends for any reason (gap closed, open set
 * exhausted, node or time limit). lb is a rigorous lower bound. res is host
 * memory. */
kc_status kc_solve(kc_handle *h, const kc_points *pts, const kc_opts *opts, kc_result *res);

#ifdef __cplusplus
}
#endif
#endif /* KC_H */
