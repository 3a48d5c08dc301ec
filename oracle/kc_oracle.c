/*
 * kc_oracle.c -- plain, serial, fp64 CPU oracle (test infrastructure only; see
 * kc_oracle.h). Every function follows the passage of the paper it cites, in
 * the paper's order of steps, with plain loops and no blocking or reordering.
 */
#include "kc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- primitives */

double kco_point_box_min_dist2(const double *x, const double *lo, const double *hi, int d) {
  /* Section 3.1: the minimiser of ||x - mu||^2 over the box is, per attribute,
   * mid{lo_a, x_a, hi_a}. */
  double s = 0.0;
  for (int a = 0; a < d; ++a) {
    double c = x[a];
    if (c < lo[a]) c = lo[a];
    if (c > hi[a]) c = hi[a];
    double t = x[a] - c;
    s += t * t;
  }
  return s;
}

double kco_point_box_max_dist2(const double *x, const double *lo, const double *hi, int d) {
  /* Section 4.2.1: the maximiser is, per attribute, lo_a if |lo_a - x_a| >
   * |hi_a - x_a|, else hi_a. */
  double s = 0.0;
  for (int a = 0; a < d; ++a) {
    double tl = fabs(lo[a] - x[a]);
    double th = fabs(hi[a] - x[a]);
    double t = tl > th ? tl : th;
    s += t * t;
  }
  return s;
}

double kco_dist2(const double *x, const double *y, int d) {
  double s = 0.0;
  for (int a = 0; a < d; ++a) {
    double t = x[a] - y[a];
    s += t * t;
  }
  return s;
}

static int in_box(const double *x, const double *lo, const double *hi, int d) {
  for (int a = 0; a < d; ++a)
    if (!(lo[a] <= x[a] && x[a] <= hi[a])) return 0;
  return 1;
}

/* ------------------------------------------------------------- node bounds */

void kco_lower_bound(const double *X, int64_t n, int d, int32_t n_nodes,
                     const int32_t *box_off, const double *lo, const double *hi,
                     double *lb, int64_t *argmax) {
  /* Eq (10): beta(M) = max_s beta_s(M); eq (11): beta_s(M) = min_k beta_s^k. */
  for (int32_t m = 0; m < n_nodes; ++m) {
    double best = -1.0;
    int64_t arg = -1;
    for (int64_t s = 0; s < n; ++s) {
      const double *x = X + s * d;
      double bs = INFINITY;
      for (int32_t b = box_off[m]; b < box_off[m + 1]; ++b) {
        double v = kco_point_box_min_dist2(x, lo + (int64_t)b * d, hi + (int64_t)b * d, d);
        if (v < bs) bs = v;
      }
      if (bs > best) {
        best = bs;
        arg = s;
      }
    }
    lb[m] = best;
    argmax[m] = arg;
  }
}

void kco_candidates(const double *X, int64_t n, int d, int32_t n_boxes,
                    const double *lo, const double *hi, int64_t *cand) {
  /* Section 3.2: for each cluster, the sample closest to the middle point of
   * M^k, taken among the samples in X cap M^k so the centers stay feasible. */
  double mid[64];
  for (int32_t b = 0; b < n_boxes; ++b) {
    const double *l = lo + (int64_t)b * d, *h = hi + (int64_t)b * d;
    for (int a = 0; a < d; ++a) mid[a] = 0.5 * (l[a] + h[a]);
    double best = INFINITY;
    int64_t arg = -1;
    for (int64_t s = 0; s < n; ++s) {
      const double *x = X + s * d;
      if (!in_box(x, l, h, d)) continue;
      double v = kco_dist2(x, mid, d);
      if (v < best) {
        best = v;
        arg = s;
      }
    }
    cand[b] = arg;
  }
}

void kco_objective(const double *X, int64_t n, int d, int32_t n_sets, int k,
                   const double *centers, double *obj, int64_t *argmax) {
  /* Eq (12): alpha = max_s min_k ||x_s - mu_hat^k||^2 (eq (1) at fixed centers). */
  for (int32_t c = 0; c < n_sets; ++c) {
    const double *C = centers + (int64_t)c * k * d;
    double best = -1.0;
    int64_t arg = -1;
    for (int64_t s = 0; s < n; ++s) {
      const double *x = X + s * d;
      double q = INFINITY;
      for (int j = 0; j < k; ++j) {
        double v = kco_dist2(x, C + (int64_t)j * d, d);
        if (v < q) q = v;
      }
      if (q > best) {
        best = q;
        arg = s;
      }
    }
    obj[c] = best;
    argmax[c] = arg;
  }
}

/* ------------------------------------------------ assignment and tightening */

int64_t kco_tighten_node(const double *X, int64_t n, int d, int k,
                         const double *lo, const double *hi, double alpha,
                         const int32_t *ref_off, const double *ref,
                         double *bb_lo, double *bb_hi, int64_t *n_in,
                         double *asg_min, double *asg_max, int64_t *n_asg,
                         int64_t *asg_far, int8_t *labels) {
  int64_t n_excluded = 0;
  double far_d[KCO_MAX_K];
  int all_have_refs = 1;
  for (int j = 0; j < k; ++j)
    if (ref_off[j + 1] <= ref_off[j]) all_have_refs = 0;
  for (int j = 0; j < k; ++j) {
    n_in[j] = 0;
    n_asg[j] = 0;
    far_d[j] = -1.0;
    if (asg_far) asg_far[j] = -1;
    for (int a = 0; a < d; ++a) {
      bb_lo[j * d + a] = INFINITY;
      bb_hi[j * d + a] = -INFINITY;
      asg_min[j * d + a] = INFINITY;
      asg_max[j * d + a] = -INFINITY;
    }
  }
  for (int64_t s = 0; s < n; ++s) {
    const double *x = X + s * d;
    int label = -1;

    /* Algorithm 3, center-based assignment (Section 4.1.1, Lemma 1): beta_s^k
     * > alpha rules cluster k out; if every cluster but k' is ruled out, s
     * belongs to k'. */
    int n_out = 0, keep = -1;
    for (int j = 0; j < k; ++j) {
      double b = kco_point_box_min_dist2(x, lo + j * d, hi + j * d, d);
      if (b > alpha)
        ++n_out;
      else
        keep = j;
    }
    if (n_out == k) {
      label = -2;
      ++n_excluded;
    } else if (n_out == k - 1) {
      label = keep;
    }

    /* Algorithm 3, sample-based assignment (Lemma 2), only for samples still
     * unassigned and only when every cluster has an assigned sample: a sample
     * farther than 4 alpha from an assigned sample of cluster j is not in j. */
    if (label == -1 && all_have_refs) {
      int n_far = 0, rest = -1;
      for (int j = 0; j < k; ++j) {
        int far = 0;
        for (int32_t r = ref_off[j]; r < ref_off[j + 1]; ++r)
          if (kco_dist2(x, ref + (int64_t)r * d, d) > 4.0 * alpha) far = 1;
        if (far)
          ++n_far;
        else
          rest = j;
      }
      if (n_far == k - 1) label = rest;
    }

    if (labels) labels[s] = (int8_t)label;
    if (label >= 0) {
      ++n_asg[label];
      for (int a = 0; a < d; ++a) {
        if (x[a] < asg_min[label * d + a]) asg_min[label * d + a] = x[a];
        if (x[a] > asg_max[label * d + a]) asg_max[label * d + a] = x[a];
      }
      /* the assigned sample farthest from the midpoint of its cluster's box */
      double dm = 0.0;
      for (int a = 0; a < d; ++a) {
        double t = x[a] - 0.5 * (lo[label * d + a] + hi[label * d + a]);
        dm += t * t;
      }
      if (dm > far_d[label]) {
        far_d[label] = dm;
        if (asg_far) asg_far[label] = s;
      }
    }

    /* Section 4.1.2, ball-based tightening with the "centers on samples"
     * constraint: S_+^k = samples in M^k within sqrt(alpha) of every ref. */
    for (int j = 0; j < k; ++j) {
      if (!in_box(x, lo + j * d, hi + j * d, d)) continue;
      int inside = 1;
      for (int32_t r = ref_off[j]; r < ref_off[j + 1]; ++r)
        if (kco_dist2(x, ref + (int64_t)r * d, d) > alpha) inside = 0;
      if (!inside) continue;
      ++n_in[j];
      for (int a = 0; a < d; ++a) {
        if (x[a] < bb_lo[j * d + a]) bb_lo[j * d + a] = x[a];
        if (x[a] > bb_hi[j * d + a]) bb_hi[j * d + a] = x[a];
      }
    }
  }
  return n_excluded;
}

int kco_tightened_box(int d, int k, const double *lo, const double *hi, double alpha,
                      const int32_t *ref_off, const double *ref,
                      const double *bb_lo, const double *bb_hi, const int64_t *n_in,
                      const double *asg_min, const double *asg_max, const int64_t *n_asg,
                      double *lo_out, double *hi_out) {
  double sa = sqrt(alpha);
  int infeasible = 0;
  for (int j = 0; j < k; ++j) {
    if (n_in[j] == 0) infeasible = 1;
    for (int a = 0; a < d; ++a) {
      /* "centers on samples": the bounding box of S_+^k. */
      double L = lo[j * d + a], H = hi[j * d + a];
      if (bb_lo[j * d + a] > L) L = bb_lo[j * d + a];
      if (bb_hi[j * d + a] < H) H = bb_hi[j * d + a];
      /* Box-based tightening: mu^k lies in [x_j - sqrt(alpha), x_j + sqrt(alpha)]
       * for every sample assigned to k (assigned samples and refs). */
      double amax = -INFINITY, amin = INFINITY;
      if (n_asg[j] > 0) {
        amax = asg_max[j * d + a];
        amin = asg_min[j * d + a];
      }
      for (int32_t r = ref_off[j]; r < ref_off[j + 1]; ++r) {
        double v = ref[(int64_t)r * d + a];
        if (v > amax) amax = v;
        if (v < amin) amin = v;
      }
      if (amax - sa > L) L = amax - sa;
      if (amin + sa < H) H = amin + sa;
      lo_out[j * d + a] = L;
      hi_out[j * d + a] = H;
      if (L > H) infeasible = 1;
    }
  }
  return infeasible;
}

int kco_symmetry(int d, int k, double *lo, double *hi) {
  /* mu_1^1 <= mu_1^2 <= ... <= mu_1^K on the first attribute. */
  for (int j = 1; j < k; ++j)
    if (lo[(j - 1) * d] > lo[j * d]) lo[j * d] = lo[(j - 1) * d];
  for (int j = k - 2; j >= 0; --j)
    if (hi[(j + 1) * d] < hi[j * d]) hi[j * d] = hi[(j + 1) * d];
  for (int j = 0; j < k; ++j)
    if (lo[j * d] > hi[j * d]) return 1;
  return 0;
}

/* ------------------------------------------------------- sample reduction */

void kco_reduce_flags(const double *X, int64_t n, int d, int32_t n_nodes,
                      const int32_t *box_off, const double *lo, const double *hi,
                      const int32_t *ref_off, const double *ref,
                      double beta, double alpha, uint8_t *keep) {
  for (int64_t s = 0; s < n; ++s) {
    const double *x = X + s * d;
    int redundant_everywhere = 1;
    for (int32_t m = 0; m < n_nodes && redundant_everywhere; ++m) {
      /* Section 4.2.1: redundant for lower bounding if alpha_s(M) < beta. */
      double as = INFINITY;
      for (int32_t b = box_off[m]; b < box_off[m + 1]; ++b) {
        double v = kco_point_box_max_dist2(x, lo + (int64_t)b * d, hi + (int64_t)b * d, d);
        if (v < as) as = v;
      }
      int lb_red = as < beta;
      /* Section 4.2.2: redundant for upper bounding if, for every cluster, x is
       * outside M^k or farther than alpha from a sample assigned to k. */
      int ub_red = 1;
      for (int32_t b = box_off[m]; b < box_off[m + 1]; ++b) {
        if (!in_box(x, lo + (int64_t)b * d, hi + (int64_t)b * d, d)) continue;
        int far = 0;
        for (int32_t r = ref_off[b]; r < ref_off[b + 1]; ++r)
          if (kco_dist2(x, ref + (int64_t)r * d, d) > alpha) far = 1;
        if (!far) ub_red = 0;
      }
      if (!(lb_red && ub_red)) redundant_everywhere = 0;
    }
    keep[s] = (uint8_t)!redundant_everywhere;
  }
}

/* ------------------------------------------------------------------- FFT */

void kco_fft(const double *X, int64_t n, int d, int k, int64_t s0, int64_t *T) {
  /* Algorithm 2 with d(x, T) = min_{t in T} ||x - t||^2. */
  T[0] = s0;
  for (int j = 1; j < k; ++j) {
    double best = -1.0;
    int64_t arg = 0;
    for (int64_t s = 0; s < n; ++s) {
      double q = INFINITY;
      for (int t = 0; t < j; ++t) {
        double v = kco_dist2(X + s * d, X + T[t] * d, d);
        if (v < q) q = v;
      }
      if (q > best) {
        best = q;
        arg = s;
      }
    }
    T[j] = arg;
  }
}

/* ------------------------------------------------------------ brute force */

void kco_brute_force(const double *X, int64_t n, int d, int k, double *best, int64_t *ids) {
  /* Eq (1) by enumeration of every k-subset in lexicographic order. A subset
   * is abandoned as soon as its running maximum reaches the best value found,
   * which cannot change the minimum or the first subset attaining it. */
  double *dm = NULL;
  if (n <= 4096) {
    dm = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j < n; ++j) dm[i * n + j] = kco_dist2(X + i * d, X + j * d, d);
  }
  int64_t c[KCO_MAX_K];
  for (int j = 0; j < k; ++j) c[j] = j;
  *best = INFINITY;
  for (int j = 0; j < k; ++j) ids[j] = j;
  for (;;) {
    double worst = -1.0;
    for (int64_t s = 0; s < n && worst < *best; ++s) {
      double q = INFINITY;
      for (int j = 0; j < k; ++j) {
        double v = dm ? dm[c[j] * n + s] : kco_dist2(X + s * d, X + c[j] * d, d);
        if (v < q) q = v;
      }
      if (q > worst) worst = q;
    }
    if (worst < *best) {
      *best = worst;
      for (int j = 0; j < k; ++j) ids[j] = c[j];
    }
    int j = k - 1;
    while (j >= 0 && c[j] == n - k + j) --j;
    if (j < 0) break;
    ++c[j];
    for (int t = j + 1; t < k; ++t) c[t] = c[t - 1] + 1;
  }
  free(dm);
}

/* --------------------------------------------------------- branch and bound */

/* A node: K boxes, its lower bound, and the samples known to belong to each
 * cluster inside it (refs: the seeds and samples assigned at its ancestors). */
typedef struct {
  double *lo, *hi; /* k*d each */
  double lb;
  int64_t id;
  int32_t roff[KCO_MAX_K + 1];
  double *ref;     /* [roff[k]][d] */
  int64_t *rid;    /* original ids of the refs */
} onode;

typedef struct {
  onode *v;
  int64_t n, cap;
} oset;

static onode node_new(int k, int d, const double *lo, const double *hi, double lb, int64_t id,
                      const int32_t *roff, const double *ref, const int64_t *rid) {
  onode m;
  m.lo = (double *)malloc(sizeof(double) * k * d);
  m.hi = (double *)malloc(sizeof(double) * k * d);
  memcpy(m.lo, lo, sizeof(double) * k * d);
  memcpy(m.hi, hi, sizeof(double) * k * d);
  m.lb = lb;
  m.id = id;
  memcpy(m.roff, roff, sizeof(int32_t) * (k + 1));
  int32_t nr = roff[k];
  m.ref = (double *)malloc(sizeof(double) * (nr > 0 ? nr : 1) * d);
  m.rid = (int64_t *)malloc(sizeof(int64_t) * (nr > 0 ? nr : 1));
  if (nr > 0) {
    memcpy(m.ref, ref, sizeof(double) * nr * d);
    memcpy(m.rid, rid, sizeof(int64_t) * nr);
  }
  return m;
}

static void node_free(onode *m) {
  free(m->lo);
  free(m->hi);
  free(m->ref);
  free(m->rid);
}

static void set_push(oset *S, onode m) {
  if (S->n == S->cap) {
    S->cap = S->cap ? 2 * S->cap : 64;
    S->v = (onode *)realloc(S->v, sizeof(onode) * S->cap);
  }
  S->v[S->n++] = m;
}

/* Node selection (Algorithm 1): the open node of least lower bound; ties go
 * to the node created first. */
static onode set_pop_min(oset *S) {
  int64_t bi = 0;
  for (int64_t i = 1; i < S->n; ++i)
    if (S->v[i].lb < S->v[bi].lb || (S->v[i].lb == S->v[bi].lb && S->v[i].id < S->v[bi].id)) bi = i;
  onode m = S->v[bi];
  S->v[bi] = S->v[S->n - 1];
  --S->n;
  return m;
}

static void set_prune(oset *S, double alpha) {
  int64_t w = 0;
  for (int64_t i = 0; i < S->n; ++i) {
    if (S->v[i].lb >= alpha)
      node_free(&S->v[i]);
    else
      S->v[w++] = S->v[i];
  }
  S->n = w;
}

/* The children's refs: the parent's refs of each cluster, then the sample the
 * parent's tightening assigned to the cluster farthest from its box midpoint,
 * unless already present or the cluster holds max_refs refs. */
static void child_refs(int k, int d, const onode *M, const int64_t *far, const double *X,
                       const int64_t *orig, int max_refs, int32_t *roff, double *ref, int64_t *rid) {
  int32_t w = 0;
  for (int j = 0; j < k; ++j) {
    roff[j] = w;
    for (int32_t r = M->roff[j]; r < M->roff[j + 1]; ++r) {
      memcpy(ref + (size_t)w * d, M->ref + (size_t)r * d, sizeof(double) * d);
      rid[w++] = M->rid[r];
    }
    if (far && far[j] >= 0 && w - roff[j] < max_refs) {
      int dup = 0;
      for (int32_t r = roff[j]; r < w; ++r)
        if (rid[r] == orig[far[j]]) dup = 1;
      if (!dup) {
        memcpy(ref + (size_t)w * d, X + far[j] * d, sizeof(double) * d);
        rid[w++] = orig[far[j]];
      }
    }
  }
  roff[k] = w;
}

int kco_solve(const double *X0, int64_t n0, int d, const kco_opts *opt, kco_result *res) {
  const int k = opt->k;
  if (k < 1 || k > KCO_MAX_K || n0 < k || d < 1 || d > 64) return -1;
  memset(res, 0, sizeof(*res));
  const int max_refs = opt->max_refs > 0 ? opt->max_refs : 1;

  /* The working dataset shrinks under sample reduction; orig maps back. */
  double *X = (double *)malloc(sizeof(double) * (size_t)n0 * d);
  int64_t *orig = (int64_t *)malloc(sizeof(int64_t) * (size_t)n0);
  memcpy(X, X0, sizeof(double) * (size_t)n0 * d);
  for (int64_t s = 0; s < n0; ++s) orig[s] = s;
  int64_t n = n0;

  /* Root region M0 (Section 2.1): per attribute the data range, for every k. */
  double *lo0 = (double *)malloc(sizeof(double) * k * d);
  double *hi0 = (double *)malloc(sizeof(double) * k * d);
  for (int a = 0; a < d; ++a) {
    double mn = X[a], mx = X[a];
    for (int64_t s = 1; s < n; ++s) {
      if (X[s * d + a] < mn) mn = X[s * d + a];
      if (X[s * d + a] > mx) mx = X[s * d + a];
    }
    for (int j = 0; j < k; ++j) {
      lo0[j * d + a] = mn;
      hi0[j * d + a] = mx;
    }
  }

  /* Root upper bound by farthest first traversal (Algorithm 2). */
  int64_t T[KCO_MAX_K];
  kco_fft(X, n, d, k, opt->fft_start, T);
  double *cent = (double *)malloc(sizeof(double) * k * d);
  for (int j = 0; j < k; ++j) memcpy(cent + j * d, X + T[j] * d, sizeof(double) * d);
  double alpha;
  int64_t am;
  kco_objective(X, n, d, 1, k, cent, &alpha, &am);
  res->fft_obj = alpha;
  for (int j = 0; j < k; ++j) res->centers[j] = T[j];

  /* K farthest initial seeds (Section 4.1.1): pairwise farther than 4 alpha
   * means the FFT points lie in distinct clusters; they become the first refs. */
  int seeds = 0;
  if (opt->use_seeds && opt->use_bt && k > 1) {
    seeds = 1;
    for (int i = 0; i < k; ++i)
      for (int j = i + 1; j < k; ++j)
        if (!(kco_dist2(X + T[i] * d, X + T[j] * d, d) > 4.0 * alpha)) seeds = 0;
  }
  res->seeds_found = seeds;
  const int grow_refs = opt->use_bt && opt->max_refs > 0;
  const size_t rcap = (size_t)k * (max_refs + 1);
  int32_t roff[KCO_MAX_K + 1];
  double *ref = (double *)malloc(sizeof(double) * rcap * d);
  int64_t *rid = (int64_t *)malloc(sizeof(int64_t) * rcap);
  for (int j = 0; j <= k; ++j) roff[j] = seeds ? j : 0;
  if (seeds)
    for (int j = 0; j < k; ++j) {
      memcpy(ref + j * d, X + T[j] * d, sizeof(double) * d);
      rid[j] = T[j];
    }
  /* Symmetry breaking (Section 4.1.3) only when no seeds were found. */
  const int symmetry = !seeds && opt->use_bt;

  oset open = {0};
  int64_t next_id = 0;
  set_push(&open, node_new(k, d, lo0, hi0, 0.0, next_id++, roff, ref, rid));

  double *lo = (double *)malloc(sizeof(double) * k * d), *hi = (double *)malloc(sizeof(double) * k * d);
  double *bbl = (double *)malloc(sizeof(double) * k * d), *bbh = (double *)malloc(sizeof(double) * k * d);
  double *amn = (double *)malloc(sizeof(double) * k * d), *amx = (double *)malloc(sizeof(double) * k * d);
  double *clo = (double *)malloc(sizeof(double) * k * d), *chi = (double *)malloc(sizeof(double) * k * d);
  int64_t nin[KCO_MAX_K], nasg[KCO_MAX_K], cand[KCO_MAX_K], far[KCO_MAX_K];
  int32_t off2[2] = {0, k};
  int32_t zero_off[KCO_MAX_K + 1];
  memset(zero_off, 0, sizeof(zero_off));
  int64_t it = 0;
  res->status = 0;

  while (open.n > 0) {
    if (opt->max_nodes > 0 && it >= opt->max_nodes) {
      res->status = 1;
      break;
    }
    /* Node selection. */
    onode M = set_pop_min(&open);
    if (M.lb >= alpha) { /* fathomed by the incumbent */
      node_free(&M);
      continue;
    }
    ++it;

    /* Bounds tightening (Algorithms 3 and 4) with the node's refs. Without the
     * acceleration techniques only the "centers on samples" box is formed
     * (infinite alpha, no refs), which the finite-termination argument of
     * Section 5 needs. */
    double a_bt = opt->use_bt ? alpha : INFINITY;
    const int32_t *mroff = opt->use_bt ? M.roff : zero_off;
    int64_t n_ex = kco_tighten_node(X, n, d, k, M.lo, M.hi, a_bt, mroff, M.ref, bbl, bbh, nin, amn,
                                    amx, nasg, far, NULL);
    int infeasible = kco_tightened_box(d, k, M.lo, M.hi, a_bt, mroff, M.ref, bbl, bbh, nin, amn, amx,
                                       nasg, lo, hi);
    if (!infeasible && symmetry) infeasible = kco_symmetry(d, k, lo, hi);
    if (n_ex > 0 || infeasible) {
      node_free(&M);
      continue;
    }
    memcpy(M.lo, lo, sizeof(double) * k * d);
    memcpy(M.hi, hi, sizeof(double) * k * d);
    /* refs the children inherit (computed before any deletion moves samples) */
    int32_t croff[KCO_MAX_K + 1];
    double *cref = (double *)malloc(sizeof(double) * rcap * d);
    int64_t *crid = (int64_t *)malloc(sizeof(int64_t) * rcap);
    child_refs(k, d, &M, grow_refs ? far : NULL, X, orig, max_refs, croff, cref, crid);

    /* Sample reduction every i_sr iterations (Algorithm 5) over every node:
     * the open set and the node in hand, each box with its cluster's refs. */
    if (opt->i_sr > 0 && it % opt->i_sr == 0) {
      int32_t nn = (int32_t)open.n + 1;
      int32_t *boff = (int32_t *)malloc(sizeof(int32_t) * (nn + 1));
      double *blo = (double *)malloc(sizeof(double) * (size_t)nn * k * d);
      double *bhi = (double *)malloc(sizeof(double) * (size_t)nn * k * d);
      int32_t *rof = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nn * k + 1));
      double *rr = (double *)malloc(sizeof(double) * ((size_t)nn * rcap + 1) * d);
      double beta = M.lb;
      int32_t nr = 0;
      rof[0] = 0;
      for (int32_t m = 0; m < nn; ++m) {
        const onode *P = m < nn - 1 ? &open.v[m] : &M;
        if (P->lb < beta) beta = P->lb;
        boff[m] = m * k;
        memcpy(blo + (size_t)m * k * d, P->lo, sizeof(double) * k * d);
        memcpy(bhi + (size_t)m * k * d, P->hi, sizeof(double) * k * d);
        for (int j = 0; j < k; ++j) {
          if (opt->use_bt)
            for (int32_t r = P->roff[j]; r < P->roff[j + 1]; ++r)
              memcpy(rr + (size_t)(nr++) * d, P->ref + (size_t)r * d, sizeof(double) * d);
          rof[m * k + j + 1] = nr;
        }
      }
      boff[nn] = nn * k;
      uint8_t *keep = (uint8_t *)malloc((size_t)n);
      kco_reduce_flags(X, n, d, nn, boff, blo, bhi, rof, rr, beta, alpha, keep);
      int64_t w = 0;
      for (int64_t s = 0; s < n; ++s)
        if (keep[s]) {
          if (w != s) {
            memmove(X + w * d, X + s * d, sizeof(double) * d);
            orig[w] = orig[s];
          }
          ++w;
        }
      n = w;
      free(keep);
      free(rr);
      free(rof);
      free(bhi);
      free(blo);
      free(boff);
    }

    /* Branch if some box still holds more than one distinct sample, i.e. is
     * not a single point after the "centers on samples" tightening. */
    int bk = -1, ba = -1;
    double bw = 0.0;
    for (int j = 0; j < k; ++j)
      for (int a = 0; a < d; ++a) {
        double w = M.hi[j * d + a] - M.lo[j * d + a];
        if (w > bw) {
          bw = w;
          bk = j;
          ba = a;
        }
      }
    if (bk < 0) {
      /* Every box is one point: the node's centers are fixed; evaluate them. */
      kco_candidates(X, n, d, k, M.lo, M.hi, cand);
      int ok = 1;
      for (int j = 0; j < k; ++j)
        if (cand[j] < 0) ok = 0;
      if (ok) {
        for (int j = 0; j < k; ++j) memcpy(cent + j * d, X + cand[j] * d, sizeof(double) * d);
        double ub;
        kco_objective(X, n, d, 1, k, cent, &ub, &am);
        if (ub < alpha) {
          alpha = ub;
          for (int j = 0; j < k; ++j) res->centers[j] = orig[cand[j]];
          set_prune(&open, alpha);
        }
      }
      free(cref);
      free(crid);
      node_free(&M);
      continue;
    }

    /* Max-range branching at the midpoint (Section 3.3). */
    double mid = 0.5 * (M.lo[bk * d + ba] + M.hi[bk * d + ba]);
    for (int side = 0; side < 2; ++side) {
      memcpy(clo, M.lo, sizeof(double) * k * d);
      memcpy(chi, M.hi, sizeof(double) * k * d);
      if (side == 0)
        chi[bk * d + ba] = mid;
      else
        clo[bk * d + ba] = mid;
      if (symmetry && kco_symmetry(d, k, clo, chi)) continue;
      /* Bounding the child: candidate centers, emptiness, LB and UB. */
      kco_candidates(X, n, d, k, clo, chi, cand);
      int empty = 0;
      for (int j = 0; j < k; ++j)
        if (cand[j] < 0) empty = 1;
      if (empty) continue;
      double blb;
      int64_t barg;
      kco_lower_bound(X, n, d, 1, off2, clo, chi, &blb, &barg);
      double clb = blb > M.lb ? blb : M.lb;
      for (int j = 0; j < k; ++j) memcpy(cent + j * d, X + cand[j] * d, sizeof(double) * d);
      double ub;
      kco_objective(X, n, d, 1, k, cent, &ub, &am);
      if (ub < alpha) {
        alpha = ub;
        for (int j = 0; j < k; ++j) res->centers[j] = orig[cand[j]];
      }
      if (clb < alpha) set_push(&open, node_new(k, d, clo, chi, clb, next_id++, croff, cref, crid));
    }
    free(cref);
    free(crid);
    set_prune(&open, alpha);
    node_free(&M);

    if (open.n > 0 && opt->eps > 0.0) {
      double glb = open.v[0].lb;
      for (int64_t i = 1; i < open.n; ++i)
        if (open.v[i].lb < glb) glb = open.v[i].lb;
      if ((alpha - glb) <= opt->eps * alpha) break;
    }
  }

  double glb = alpha;
  for (int64_t i = 0; i < open.n; ++i)
    if (open.v[i].lb < glb) glb = open.v[i].lb;
  res->obj = alpha;
  res->lb = glb;
  res->nodes = it;
  res->n_active = n;
  for (int64_t i = 0; i < open.n; ++i) node_free(&open.v[i]);
  free(open.v);
  free(lo);
  free(hi);
  free(bbl);
  free(bbh);
  free(amn);
  free(amx);
  free(clo);
  free(chi);
  free(ref);
  free(rid);
  free(cent);
  free(lo0);
  free(hi0);
  free(orig);
  free(X);
  return 0;
}
