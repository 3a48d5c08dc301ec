// kc_solve.cpp -- host branch and bound (Algorithm 1) over the libkc calls.
//
// Per pass: pop up to `batch` open nodes of least lower bound; one kc_tighten
// launch gives the assignment / tightening aggregates of all of them
// (Algorithms 3-4) and the host forms the tightened boxes; every `i_sr` passes
// kc_reduce deletes the samples redundant in every open node (Algorithm 5),
// and with node_sr a node may get a sample set of its own from a reduction
// over itself alone, which its subtree inherits (nodes sharing samples are
// launched together); each surviving node is split (max-range rule of Section 3.3, or the learned
// rule) and one kc_lower_bound launch bounds all children and returns their
// Section 3.2 candidates; one kc_objective launch screens the candidates in
// float32 (rounded up), and the best set's rigorous float32 bound becomes the
// incumbent bound that prunes; its float64 objective over the original
// samples is taken once, when the search ends (a later improvement always
// beats an earlier one, so only the last needs it). Nodes are pruned when their rigorous lower bound reaches
// the incumbent, and every node that leaves the tree records the bound it
// leaves behind, so the final lower bound is rigorous too.
//
// Host <-> device traffic per phase is one packed upload and one packed
// download through a pinned staging arena; the coordinates of candidates and
// new refs are gathered on the device, so a pass synchronises twice (after
// the tightening phase and after the bounding phase), plus once for a
// sample reduction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <vector>

#include "kc_internal.h"

// Host float64 arithmetic stays unfused so that distance sums round exactly as
// written (the seeds test compares them with 4 alpha).
#pragma clang fp contract(off)

namespace {

constexpr int NFEAT = 32;
// The learned rule and the strong-branching labels consider only the sides at
// least this fraction of the node's widest side: every split still halves a
// side within a factor 2 of the widest, so the subdivision stays exhaustive
// (the widest side halves at least every K*D splits along a path).
constexpr double kWideFrac = 0.5;

// Pinned host buffer with a device mirror, bump-allocated per phase: offsets
// are taken first, then reserve() sizes both sides, then the host side is
// filled and moved with one copy.
struct Arena {
  char *h = nullptr, *d = nullptr;
  size_t cap = 0, used = 0;
  ~Arena() {
    if (h) (void)hipHostFree(h);
    if (d) (void)hipFree(d);
  }
  void reset() { used = 0; }
  size_t take(size_t bytes) {
    const size_t o = (used + 255) & ~(size_t)255;
    used = o + bytes;
    return o;
  }
  bool reserve() {
    if (used <= cap) return true;
    if (h || d) {
      (void)hipDeviceSynchronize();  // earlier work may still use the old buffers
      if (h) (void)hipHostFree(h);
      if (d) (void)hipFree(d);
      h = d = nullptr;
      cap = 0;
    }
    const size_t nb = used + used / 2 + 4096;
    if (hipHostMalloc((void **)&h, nb, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      h = nullptr;
      return false;
    }
    if (hipMalloc((void **)&d, nb) != hipSuccess) {
      (void)hipGetLastError();
      d = nullptr;
      return false;
    }
    cap = nb;
    return true;
  }
  template <class T>
  T *hp(size_t o) const {
    return (T *)(h + o);
  }
  template <class T>
  T *dp(size_t o) const {
    return (T *)(d + o);
  }
};

struct DevBuf {
  void *p = nullptr;
  size_t cap = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  bool ensure(size_t bytes) {
    if (bytes <= cap) return true;
    if (p) {
      (void)hipDeviceSynchronize();
      (void)hipFree(p);
      p = nullptr;
      cap = 0;
    }
    const size_t nb = bytes + 256;
    if (hipMalloc(&p, nb) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      return false;
    }
    cap = nb;
    return true;
  }
  template <class T>
  T *as() const {
    return (T *)p;
  }
};

// The samples one subtree still needs: what a sample reduction over one node
// with that node's own lower bound kept (Section 4.2: a sample redundant in a
// node stays redundant in every node below it). The node's descendants share
// it; when the last one leaves the tree the buffers go back to the driver's
// pool for the next set.
struct SampleSet {
  DevBuf x, ids;                 // [D][ld] coordinates, [n] original ids
  int64_t n = 0, ld = 0;
};

struct Node {
  std::vector<float> lo, hi;     // K*D (row k: lo[k*D + a])
  double lb = 0.0;               // rigorous lower bound
  double parent_lb = 0.0;
  int64_t id = 0;
  int depth = 0;
  int split_k = -1, split_a = -1, side = -1;
  std::vector<uint8_t> nsplit;   // K*D: splits of (k,a) on the path
  float xstar[16] = {0};         // sample attaining the node's lower bound
  // samples known to belong to each cluster inside the node (seeds and the
  // samples assigned at its ancestors): cluster k owns rows roff[k]..roff[k+1]-1
  std::vector<int32_t> roff;
  std::vector<float> ref;        // [rows][D]
  std::vector<int64_t> rid;      // original sample ids
  // refs found by this node's tightening, handed to its children
  std::vector<float> new_ref;    // [K][D]
  std::vector<int64_t> new_rid;  // [K], -1 = none
  // samples of the subtree (null: the driver's active samples), and how many
  // more generations wait before the next one-node reduction is tried
  std::shared_ptr<SampleSet> ss;
  uint8_t sr_wait = 0, sr_backoff = 0;
};

struct HeapCmp {
  bool operator()(const Node *a, const Node *b) const {
    return a->lb > b->lb || (a->lb == b->lb && a->id > b->id);
  }
};

inline double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Splits [lo, hi] (lo < hi) into [lo, m] and [next(m), hi]: together they hold
// every float32 of [lo, hi], and centers are float32 samples.
void split_interval(float lo, float hi, float *l_hi, float *r_lo) {
  float m = kc_round_down_f32(0.5 * ((double)lo + (double)hi));
  if (m >= hi) m = nextafterf(hi, -INFINITY);
  if (m < lo) m = lo;
  *l_hi = m;
  *r_lo = nextafterf(m, INFINITY);
}

struct Solver {
  kc_handle *h;
  const kc_points *X0;
  kc_opts o;
  kc_result *res;
  int K, D;
  hipStream_t st = nullptr;

  // active samples
  kc_points act;
  const uint32_t *idx = nullptr;  // active -> original (null: identity)
  DevBuf xbuf[2], ibuf[2];
  int cur = -1;

  // incumbent
  double alpha_cert = INFINITY;   // float64 objective over all samples
  double alpha_ub = INFINITY;     // valid upper bound used for pruning
  std::vector<int64_t> inc_ids;
  std::vector<float> inc_coords;
  // best set found since the last certificate (alpha_ub bounds its objective)
  bool pending = false;
  std::vector<int64_t> pend_ids;
  std::vector<float> pend_coords;
  double lb_closed = INFINITY;    // least bound among nodes that left the tree

  // root data
  std::vector<float> root_lo, root_hi;
  bool seeds = false, symmetry = false;

  std::vector<Node *> heap;
  int64_t next_id = 0, n_branched = 0;
  int sb_nodes = 0, sb_rows = 0;

  // pseudocosts per (k,a): sums and counts of relative LB gains
  std::vector<double> pc_sum[2];
  std::vector<int> pc_cnt[2];

  Arena in, out;
  double t0 = 0;
  // wall time per phase (reported with verbose)
  double t_tighten = 0, t_reduce = 0, t_branch = 0, t_bound = 0;
  int64_t sr_interval = 0, sr_runs = 0;
  int64_t trigger_calls = 0;  // reduction-trigger calls on a very large open set
  int64_t n_bounded = 0, n_bounded_pruned = 0;  // bounded nodes, and those the bound prunes
  // subtree sample sets: bytes held and the cap on them; measured cost of a
  // one-node reduction per sample of the node
  size_t set_bytes = 0, set_cap = 0;  // held by live and pooled sets
  int64_t last_pass_evals = 0;      // lower-bound + tightening evaluations of the last pass
  double nsr_keep_rate[10] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1};  // recent fraction kept per lb/alpha tenth
  int64_t n_pass = 0, nsr_last_pass = 0;
  std::vector<std::unique_ptr<SampleSet>> pool;

  Solver(kc_handle *h_, const kc_points *x, const kc_opts *op, kc_result *r)
      : h(h_), X0(x), o(*op), res(r), K(op->k), D(x->d) {
    act = *x;
  }
  ~Solver() {
    for (Node *n : heap) delete n;
    if (st) (void)hipStreamDestroy(st);
  }

  kc_status sync(const char *what) {
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return kc_fail(h, KC_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return KC_OK;
  }
  kc_status reserve() {
    if (!in.reserve() || !out.reserve()) return kc_fail(h, KC_ENOMEM, "driver staging buffers");
    return KC_OK;
  }
  kc_status upload() {
    if (in.used && hipMemcpyAsync(in.d, in.h, in.used, hipMemcpyHostToDevice, st) != hipSuccess)
      return kc_fail(h, KC_EDEVICE, "upload");
    return KC_OK;
  }
  kc_status download(const char *what) {
    if (out.used && hipMemcpyAsync(out.h, out.d, out.used, hipMemcpyDeviceToHost, st) != hipSuccess)
      return kc_fail(h, KC_EDEVICE, "download");
    return sync(what);
  }

  double prune_thr() const { return alpha_ub * (1.0 - o.eps_rel); }

  // Float64 objective over the original samples of the pending set: it
  // becomes the incumbent if it beats the certified one (it always does,
  // since its rigorous float32 bound was below every earlier bound).
  kc_status certify() {
    if (!pending) return KC_OK;
    pending = false;
    in.reset();
    out.reset();
    const size_t o_c = in.take((size_t)K * D * 4), o_v = out.take(8);
    kc_status s = reserve();
    if (s) return s;
    std::memcpy(in.hp<float>(o_c), pend_coords.data(), (size_t)K * D * 4);
    if ((s = upload())) return s;
    if ((s = kc_objective(h, X0, 1, K, in.dp<float>(o_c), 64, out.dp<double>(o_v), nullptr, st)))
      return s;
    res->passes++;
    if ((s = download("certificate"))) return s;
    const double cert = *out.hp<double>(o_v);
    if (cert < alpha_cert) {
      alpha_cert = cert;
      inc_ids = pend_ids;
      inc_coords = pend_coords;
    }
    alpha_ub = std::min(alpha_ub, alpha_cert);
    return KC_OK;
  }
  // Screening threshold of the candidates' float32 objective: a set whose
  // value v exceeds it has v (1 + rel) + eta > alpha_ub, so it cannot become
  // the incumbent, and its launch may stop early (reporting the value of some
  // sample above the threshold, still a lower bound of its objective).
  float screen_cut() const {
    if (!(alpha_ub < INFINITY)) return INFINITY;
    const double rel = kc_rel_margin(D) + 0x1p-50, eta = kc_abs_margin(D);
    const double c = (alpha_ub - eta) / (1.0 + rel) * (1.0 + 0x1p-40);
    if (!(c > 0.0)) return 0.0f;
    float f = (float)c;
    if ((double)f < c) f = std::nextafter(f, INFINITY);
    return f;
  }

  // Samples a node is bounded over: its subtree's set, else the active ones.
  kc_points pts_of(const Node *m) const {
    kc_points p = act;
    if (m->ss) {
      p.x = m->ss->x.as<float>();
      p.n = m->ss->n;
      p.ld = m->ss->ld;
    }
    return p;
  }
  const uint32_t *idx_of(const Node *m) const { return m->ss ? m->ss->ids.as<uint32_t>() : idx; }

  // Maximal runs [first, last) of consecutive nodes bounded over the same
  // samples: one launch per run.
  static std::vector<std::pair<int, int>> runs(const std::vector<Node *> &v) {
    std::vector<std::pair<int, int>> r;
    for (int i = 0; i < (int)v.size();) {
      int j = i + 1;
      while (j < (int)v.size() && v[j]->ss == v[i]->ss) ++j;
      r.push_back({i, j});
      i = j;
    }
    return r;
  }
  // Stable permutation that puts nodes sharing their samples next to each
  // other (the identity when no node has a subtree set).
  static std::vector<int> group_order(const std::vector<Node *> &v) {
    std::vector<const SampleSet *> first;
    std::vector<int> key(v.size());
    for (size_t i = 0; i < v.size(); ++i) {
      const SampleSet *p = v[i]->ss.get();
      size_t g = 0;
      while (g < first.size() && first[g] != p) ++g;
      if (g == first.size()) first.push_back(p);
      key[i] = (int)g;
    }
    std::vector<int> perm(v.size());
    for (size_t i = 0; i < v.size(); ++i) perm[i] = (int)i;
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return key[a] < key[b]; });
    return perm;
  }

  void heap_push(Node *n) {
    heap.push_back(n);
    std::push_heap(heap.begin(), heap.end(), HeapCmp());
  }
  Node *heap_pop() {
    std::pop_heap(heap.begin(), heap.end(), HeapCmp());
    Node *n = heap.back();
    heap.pop_back();
    return n;
  }
  double global_lb() const {
    double lb = lb_closed;
    if (!heap.empty()) lb = std::min(lb, heap.front()->lb);
    return std::min(lb, alpha_cert);
  }

  // Offsets of a packed node batch (boxes, optional refs) in the input arena.
  struct BoxPlan {
    size_t off, lo, hi, roff, ref;
    int nn, n_refs, max_refs;
    bool refs;
  };
  BoxPlan plan_boxes(const std::vector<const std::vector<float> *> &los,
                     const std::vector<const Node *> *ref_nodes) {
    BoxPlan P{};
    P.nn = (int)los.size();
    P.off = in.take((size_t)(P.nn + 1) * 4);
    P.lo = in.take((size_t)P.nn * K * D * 4);
    P.hi = in.take((size_t)P.nn * K * D * 4);
    P.refs = false;
    P.n_refs = 0;
    P.max_refs = 0;
    if (ref_nodes) {
      for (const Node *m : *ref_nodes)
        for (int k = 0; k < K; ++k) {
          const int c = m->roff.empty() ? 0 : m->roff[k + 1] - m->roff[k];
          P.n_refs += c;
          P.max_refs = std::max(P.max_refs, c);
        }
      P.refs = P.n_refs > 0;
      if (P.refs) {
        P.roff = in.take((size_t)(P.nn * K + 1) * 4);
        P.ref = in.take((size_t)P.n_refs * D * 4);
      }
    }
    return P;
  }
  void fill_boxes(const BoxPlan &P, const std::vector<const std::vector<float> *> &los,
                  const std::vector<const std::vector<float> *> &his,
                  const std::vector<const Node *> *ref_nodes) {
    int32_t *off = in.hp<int32_t>(P.off);
    float *lo = in.hp<float>(P.lo), *hi = in.hp<float>(P.hi);
    for (int i = 0; i < P.nn; ++i) {
      off[i] = i * K;
      std::memcpy(lo + (size_t)i * K * D, los[i]->data(), (size_t)K * D * 4);
      std::memcpy(hi + (size_t)i * K * D, his[i]->data(), (size_t)K * D * 4);
    }
    off[P.nn] = P.nn * K;
    if (P.refs) {
      int32_t *roff = in.hp<int32_t>(P.roff);
      float *ref = in.hp<float>(P.ref);
      int32_t w = 0;
      for (int i = 0; i < P.nn; ++i) {
        const Node *m = (*ref_nodes)[i];
        for (int k = 0; k < K; ++k) {
          roff[i * K + k] = w;
          const int c = m->roff.empty() ? 0 : m->roff[k + 1] - m->roff[k];
          if (c > 0) std::memcpy(ref + (size_t)w * D, m->ref.data() + (size_t)m->roff[k] * D, (size_t)c * D * 4);
          w += c;
        }
      }
      roff[P.nn * K] = w;
    }
  }
  kc_nodes dev_nodes(const BoxPlan &P) const {
    return kc_nodes{P.nn, P.nn * K, K, 0, in.dp<int32_t>(P.off), in.dp<float>(P.lo), in.dp<float>(P.hi)};
  }
  kc_refs dev_refs(const BoxPlan &P) const {
    return kc_refs{P.n_refs, P.max_refs, in.dp<int32_t>(P.roff), in.dp<float>(P.ref)};
  }

  // ---------------------------------------------------------------- root --
  kc_status root() {
    // Root region M0 (Section 2.1) as the bounding box of one all-space box.
    in.reset();
    out.reset();
    const size_t o_off = in.take(8), o_lo = in.take(D * 4), o_hi = in.take(D * 4);
    const size_t o_bl = out.take(D * 4), o_bh = out.take(D * 4), o_am = out.take(D * 4),
                 o_ax = out.take(D * 4), o_ni = out.take(4), o_na = out.take(4), o_ne = out.take(4);
    const size_t o_ids = in.take(64 * 8);
    const size_t o_coords = out.take((size_t)64 * D * 4), o_obj = out.take(8), o_oam = out.take(8);
    kc_status s = reserve();
    if (s) return s;
    int32_t *off = in.hp<int32_t>(o_off);
    off[0] = 0;
    off[1] = 1;
    for (int a = 0; a < D; ++a) {
      in.hp<float>(o_lo)[a] = -INFINITY;
      in.hp<float>(o_hi)[a] = INFINITY;
    }
    if ((s = upload())) return s;
    kc_nodes nd{1, 1, 1, 0, in.dp<int32_t>(o_off), in.dp<float>(o_lo), in.dp<float>(o_hi)};
    s = kc_tighten(h, &act, &nd, INFINITY, nullptr, out.dp<float>(o_bl), out.dp<float>(o_bh),
                   out.dp<uint32_t>(o_ni), out.dp<float>(o_am), out.dp<float>(o_ax),
                   out.dp<uint32_t>(o_na), out.dp<uint32_t>(o_ne), nullptr, nullptr, st);
    if (s) return s;
    res->passes++;
    if ((s = download("root box"))) return s;
    root_lo.assign(K * D, 0.f);
    root_hi.assign(K * D, 0.f);
    for (int k = 0; k < K; ++k)
      for (int a = 0; a < D; ++a) {
        root_lo[k * D + a] = out.hp<float>(o_bl)[a];
        root_hi[k * D + a] = out.hp<float>(o_bh)[a];
      }

    // Farthest first traversal (Algorithm 2), distances in float64.
    std::vector<int64_t> T(K);
    T[0] = o.fft_start;
    for (int j = 1; j <= K; ++j) {
      std::memcpy(in.hp<int64_t>(o_ids), T.data(), (size_t)j * 8);
      if (hipMemcpyAsync(in.dp<int64_t>(o_ids), in.hp<int64_t>(o_ids), (size_t)j * 8,
                         hipMemcpyHostToDevice, st) != hipSuccess)
        return kc_fail(h, KC_EDEVICE, "upload");
      if ((s = kc_gather(h, &act, in.dp<int64_t>(o_ids), j, nullptr, out.dp<float>(o_coords), nullptr, st)))
        return s;
      s = kc_objective(h, &act, 1, j, out.dp<float>(o_coords), 64, out.dp<double>(o_obj),
                       out.dp<int64_t>(o_oam), st);
      if (s) return s;
      res->passes++;
      if ((s = download("fft"))) return s;
      if (j < K)
        T[j] = *out.hp<int64_t>(o_oam);
      else
        alpha_cert = *out.hp<double>(o_obj);
    }
    inc_ids = T;
    inc_coords.assign(out.hp<float>(o_coords), out.hp<float>(o_coords) + K * D);
    alpha_ub = alpha_cert;
    res->fft_obj = alpha_cert;

    // K farthest initial seeds (Section 4.1.1): pairwise farther than 4 alpha.
    seeds = false;
    if (o.use_seeds && o.use_bt && K > 1) {
      seeds = true;
      for (int i = 0; i < K && seeds; ++i)
        for (int j = i + 1; j < K; ++j) {
          double dd = 0;
          for (int a = 0; a < D; ++a) {
            const double t = (double)inc_coords[i * D + a] - (double)inc_coords[j * D + a];
            dd += t * t;
          }
          if (!(dd > 4.0 * alpha_cert)) {
            seeds = false;
            break;
          }
        }
    }
    symmetry = !seeds && o.use_bt;
    res->seeds_found = seeds;

    Node *r = new Node();
    r->lo = root_lo;
    r->hi = root_hi;
    r->lb = 0.0;
    r->id = next_id++;
    r->nsplit.assign(K * D, 0);
    r->roff.assign(K + 1, 0);
    if (seeds) {
      for (int k = 0; k <= K; ++k) r->roff[k] = k;
      r->ref = inc_coords;
      r->rid = inc_ids;
    }
    if (symmetry) apply_symmetry(r->lo, r->hi);
    heap_push(r);
    for (int s2 = 0; s2 < 2; ++s2) {
      pc_sum[s2].assign(K * D, 0.0);
      pc_cnt[s2].assign(K * D, 0);
    }
    return KC_OK;
  }

  // A child's refs: its parent's refs of each cluster, then the sample the
  // parent's tightening assigned to that cluster farthest from the box
  // midpoint, unless already present or the cluster holds max_refs refs.
  void inherit_refs(const Node *p, Node *c) const {
    c->roff.assign(K + 1, 0);
    c->ref.clear();
    c->rid.clear();
    int32_t w = 0;
    for (int k = 0; k < K; ++k) {
      c->roff[k] = w;
      if (!p->roff.empty())
        for (int r = p->roff[k]; r < p->roff[k + 1]; ++r) {
          c->ref.insert(c->ref.end(), p->ref.begin() + (size_t)r * D, p->ref.begin() + (size_t)(r + 1) * D);
          c->rid.push_back(p->rid[r]);
          ++w;
        }
      if (!p->new_rid.empty() && p->new_rid[k] >= 0 && w - c->roff[k] < o.max_refs) {
        bool dup = false;
        for (int r = c->roff[k]; r < w; ++r)
          if (c->rid[r] == p->new_rid[k]) dup = true;
        if (!dup) {
          c->ref.insert(c->ref.end(), p->new_ref.begin() + (size_t)k * D, p->new_ref.begin() + (size_t)(k + 1) * D);
          c->rid.push_back(p->new_rid[k]);
          ++w;
        }
      }
    }
    c->roff[K] = w;
  }

  double max_width(const Node *m) const {
    double w = 0.0;
    for (int q = 0; q < K * D; ++q) w = std::max(w, (double)m->hi[q] - m->lo[q]);
    return w;
  }

  // Section 4.1.3: mu_1^1 <= ... <= mu_1^K on the first attribute.
  bool apply_symmetry(std::vector<float> &lo, std::vector<float> &hi) const {
    for (int k = 1; k < K; ++k) lo[k * D] = std::max(lo[k * D], lo[(k - 1) * D]);
    for (int k = K - 2; k >= 0; --k) hi[k * D] = std::min(hi[k * D], hi[(k + 1) * D]);
    for (int k = 0; k < K; ++k)
      if (lo[k * D] > hi[k * D]) return false;
    return true;
  }

  // ------------------------------------------------------------ tighten --
  struct TAgg {
    std::vector<uint32_t> nin, nasg;
  } ta;

  // Tightens every node of the batch in place (M-hat of Algorithm 4) and
  // records the refs it found for the node's children; alive[i] = 0 when the
  // node holds no solution of objective <= a_bt.
  kc_status tighten(std::vector<Node *> &batch, std::vector<char> &alive, double a_bt) {
    const int nn = (int)batch.size();
    const bool want_far = o.use_bt && o.max_refs > 0;
    in.reset();
    out.reset();
    // one launch per run of nodes sharing their samples
    const auto R = runs(batch);
    std::vector<BoxPlan> plans;
    std::vector<std::vector<const std::vector<float> *>> glo(R.size()), ghi(R.size());
    std::vector<std::vector<const Node *>> gnode(R.size());
    for (size_t g = 0; g < R.size(); ++g) {
      for (int i = R[g].first; i < R[g].second; ++i) {
        glo[g].push_back(&batch[i]->lo);
        ghi[g].push_back(&batch[i]->hi);
        gnode[g].push_back(batch[i]);
      }
      plans.push_back(plan_boxes(glo[g], o.use_bt ? &gnode[g] : nullptr));
    }
    const size_t nbd = (size_t)nn * K * D, nb = (size_t)nn * K;
    const size_t o_bl = out.take(nbd * 4), o_bh = out.take(nbd * 4), o_am = out.take(nbd * 4),
                 o_ax = out.take(nbd * 4), o_ni = out.take(nb * 4), o_na = out.take(nb * 4),
                 o_ne = out.take((size_t)nn * 4), o_far = out.take(nb * 8),
                 o_fc = out.take(nb * D * 4), o_fo = out.take(nb * 8);
    kc_status s = reserve();
    if (s) return s;
    for (size_t g = 0; g < R.size(); ++g) fill_boxes(plans[g], glo[g], ghi[g], o.use_bt ? &gnode[g] : nullptr);
    if ((s = upload())) return s;
    if (o.autotune)  // shapes new to the handle's table: sweep the tiles first
      for (size_t g = 0; g < R.size(); ++g) {
        const kc_points p = pts_of(batch[R[g].first]);
        const kc_nodes nd = dev_nodes(plans[g]);
        const kc_refs rf = dev_refs(plans[g]);
        bool tuned = false;
        (void)kc_tighten_tile(h, &p, &nd, plans[g].refs ? &rf : nullptr, &tuned);
        if (!tuned && (s = kc_autotune_tighten(h, &p, &nd, a_bt, plans[g].refs ? &rf : nullptr,
                                               nullptr, st)))
          return s;
      }
    (void)hipEventRecord(h->ev0, st);
    for (size_t g = 0; g < R.size(); ++g) {
      const size_t i0 = (size_t)R[g].first, gn = (size_t)(R[g].second - R[g].first);
      const kc_points p = pts_of(batch[i0]);
      const kc_nodes nd = dev_nodes(plans[g]);
      const kc_refs rf = dev_refs(plans[g]);
      s = kc_tighten(h, &p, &nd, a_bt, plans[g].refs ? &rf : nullptr, out.dp<float>(o_bl) + i0 * K * D,
                     out.dp<float>(o_bh) + i0 * K * D, out.dp<uint32_t>(o_ni) + i0 * K,
                     out.dp<float>(o_am) + i0 * K * D, out.dp<float>(o_ax) + i0 * K * D,
                     out.dp<uint32_t>(o_na) + i0 * K, out.dp<uint32_t>(o_ne) + i0,
                     want_far ? out.dp<int64_t>(o_far) + i0 * K : nullptr, nullptr, st);
      if (s) return s;
      res->passes++;
      res->tighten_evals += p.n * (int64_t)gn * K;
    }
    (void)hipEventRecord(h->ev1, st);
    // coordinates and original ids of the new refs, gathered before any
    // sample reduction moves the samples
    if (want_far)
      for (size_t g = 0; g < R.size(); ++g) {
        const size_t i0 = (size_t)R[g].first, gn = (size_t)(R[g].second - R[g].first);
        const kc_points p = pts_of(batch[i0]);
        if ((s = kc_gather(h, &p, out.dp<int64_t>(o_far) + i0 * K, (int)(gn * K), idx_of(batch[i0]),
                           out.dp<float>(o_fc) + i0 * K * D, out.dp<int64_t>(o_fo) + i0 * K, st)))
          return s;
      }
    if ((s = download("tighten"))) return s;
    {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, h->ev0, h->ev1);
      res->tighten_kernel_ms += ms;
    }

    const float *bbl = out.hp<float>(o_bl), *bbh = out.hp<float>(o_bh);
    const float *amn = out.hp<float>(o_am), *amx = out.hp<float>(o_ax);
    const uint32_t *nin = out.hp<uint32_t>(o_ni), *nasg = out.hp<uint32_t>(o_na);
    const uint32_t *nex = out.hp<uint32_t>(o_ne);
    const int64_t *far = out.hp<int64_t>(o_far);
    const float *fc = out.hp<float>(o_fc);
    const int64_t *fo = out.hp<int64_t>(o_fo);
    ta.nin.assign(nin, nin + nb);
    ta.nasg.assign(nasg, nasg + nb);

    const double sa = o.use_bt ? std::sqrt(a_bt) * (1.0 + 0x1p-50) : INFINITY;
    alive.assign(nn, 1);
    for (int i = 0; i < nn; ++i) {
      Node *m = batch[i];
      if (want_far) {
        m->new_ref.assign((size_t)K * D, 0.f);
        m->new_rid.assign(K, -1);
        for (int k = 0; k < K; ++k) {
          const size_t b = (size_t)i * K + k;
          if (far[b] >= 0) {
            std::memcpy(&m->new_ref[(size_t)k * D], fc + b * D, (size_t)D * 4);
            m->new_rid[k] = fo[b];
          }
        }
      }
      bool ok = nex[i] == 0;
      for (int k = 0; k < K && ok; ++k) {
        const size_t b = (size_t)i * K + k;
        if (nin[b] == 0) {
          ok = false;
          break;
        }
        for (int a = 0; a < D; ++a) {
          const size_t q = b * D + a;
          float L = std::max(m->lo[k * D + a], bbl[q]);
          float H = std::min(m->hi[k * D + a], bbh[q]);
          if (o.use_bt && std::isfinite(sa)) {
            // box-based tightening with the assigned samples and the refs
            double amax = -INFINITY, amin = INFINITY;
            if (nasg[b] > 0) {
              amax = amx[q];
              amin = amn[q];
            }
            if (!m->roff.empty())
              for (int r = m->roff[k]; r < m->roff[k + 1]; ++r) {
                amax = std::max(amax, (double)m->ref[(size_t)r * D + a]);
                amin = std::min(amin, (double)m->ref[(size_t)r * D + a]);
              }
            if (std::isfinite(amax)) L = std::max(L, kc_round_up_f32(nextafter(amax - sa, -INFINITY)));
            if (std::isfinite(amin)) H = std::min(H, kc_round_down_f32(nextafter(amin + sa, INFINITY)));
          }
          if (!(L <= H)) ok = false;
          m->lo[k * D + a] = L;
          m->hi[k * D + a] = H;
        }
      }
      if (ok && symmetry) ok = apply_symmetry(m->lo, m->hi);
      alive[i] = ok;
    }
    return KC_OK;
  }

  // ---------------------------------------------------- sample reduction --
  // Whether the reduction over the open nodes and `extra` can delete any
  // sample. A sample is LB-redundant in a node (Section 4.2.1) only if its
  // farthest-corner distance to some box is below beta, the least lower
  // bound; from any point the farthest corner of a box is at least half its
  // diagonal away, so a node none of whose boxes has a squared half-diagonal
  // below beta keeps every sample (and the reduction keeps what any node
  // keeps).
  bool can_reduce(const std::vector<Node *> &extra) {
    const double thr = prune_thr();
    // least bound among the open nodes below the threshold: the heap's front
    // (a scan of the whole heap every pass would cost more than the kernels
    // once the open set holds millions of nodes)
    double beta = !heap.empty() && heap.front()->lb < thr ? heap.front()->lb : INFINITY;
    for (const Node *m : extra) beta = std::min(beta, m->lb);
    if (!(beta > 0) || !std::isfinite(beta)) return false;
    auto small_box = [&](const Node *m) {
      for (int k = 0; k < K; ++k) {
        double r2 = 0;
        for (int a = 0; a < D; ++a) {
          const double hw = 0.5 * ((double)m->hi[k * D + a] - m->lo[k * D + a]);
          r2 += hw * hw;
        }
        if (r2 * (1.0 - 1e-12) < beta) return true;
      }
      return false;
    };
    for (const Node *m : extra)
      if (!small_box(m)) return false;
    // the least-bound nodes (the top of the heap) first: they are the likeliest
    // to keep a large box, which ends the scan of the open set at once
    for (size_t i = 0; i < heap.size() && i < 64; ++i)
      if (heap[i]->lb < thr && !small_box(heap[i])) return false;
    // a scan of a very large open set runs on every 16th call only (a
    // reduction that could already run waits a few passes; none is unsafe)
    if (heap.size() > 65536 && (++trigger_calls & 15) != 0) return false;
    for (const Node *m : heap)
      if (m->lb < thr && !small_box(m)) return false;
    return true;
  }

  // Over every open node, so the active samples stay valid for all of them;
  // a subtree set no smaller than the result is then dropped. *kept: the
  // number of samples the flags keep. When they would delete under 5%, the
  // samples stay as they are (keeping redundant samples is always valid, and
  // a compaction pass over all of them would cost more than it saves).
  kc_status reduce(const std::vector<Node *> &extra, int64_t *kept) {
    *kept = act.n;
    std::vector<const std::vector<float> *> los, his;
    std::vector<const Node *> ns;
    double beta = INFINITY;
    const double thr = prune_thr();
    for (Node *m : heap)
      if (m->lb < thr) {
        los.push_back(&m->lo);
        his.push_back(&m->hi);
        ns.push_back(m);
        beta = std::min(beta, m->lb);
      }
    for (Node *m : extra) {
      los.push_back(&m->lo);
      his.push_back(&m->hi);
      ns.push_back(m);
      beta = std::min(beta, m->lb);
    }
    if (los.empty()) return KC_OK;
    in.reset();
    out.reset();
    const BoxPlan P = plan_boxes(los, o.use_bt ? &ns : nullptr);
    const size_t o_n = out.take(8);
    kc_status s = reserve();
    if (s) return s;
    fill_boxes(P, los, his, o.use_bt ? &ns : nullptr);
    if ((s = upload())) return s;
    const int nxt = cur == 0 ? 1 : 0;
    const size_t bytes = (size_t)D * X0->ld * 4;
    if (!xbuf[nxt].ensure(bytes) || !ibuf[nxt].ensure((size_t)X0->ld * 4))
      return kc_fail(h, KC_ENOMEM, "sample buffers");
    const kc_nodes nd = dev_nodes(P);
    const kc_refs rf = dev_refs(P);
    s = kc_reduce_count(h, &act, &nd, P.refs ? &rf : nullptr, beta, alpha_ub, out.dp<int64_t>(o_n),
                        st);
    if (s) return s;
    res->passes++;
    if ((s = download("reduce"))) return s;
    const int64_t n_out = *out.hp<int64_t>(o_n);
    if (n_out < 1) return KC_OK;  // keep the previous set (nothing left to bound)
    *kept = n_out;
    if (n_out * 20 > act.n * 19) return KC_OK;
    if ((s = kc_reduce_compact(h, &act, idx, n_out, xbuf[nxt].as<float>(), ibuf[nxt].as<uint32_t>(),
                               X0->ld, st)))
      return s;
    cur = nxt;
    act.x = xbuf[cur].as<float>();
    act.n = n_out;
    act.ld = X0->ld;
    idx = ibuf[cur].as<uint32_t>();
    for (Node *m : heap)
      if (m->ss && m->ss->n >= act.n) m->ss.reset();
    for (Node *m : extra)
      if (m->ss && m->ss->n >= act.n) m->ss.reset();
    return KC_OK;
  }

  // Buffers for a subtree set of leading dimension ld: the smallest pooled
  // ones that fit (and are at most 4x the need), else new ones within the cap
  // (pooled buffers are freed first to make room). Null when over the cap.
  std::shared_ptr<SampleSet> take_set(int64_t ld) {
    const size_t need_x = (size_t)D * ld * 4, need_i = (size_t)ld * 4;
    int best = -1;
    for (int i = 0; i < (int)pool.size(); ++i) {
      const SampleSet &q = *pool[i];
      if (q.x.cap >= need_x && q.ids.cap >= need_i && q.x.cap <= 4 * need_x + 4096 &&
          (best < 0 || q.x.cap < pool[best]->x.cap))
        best = i;
    }
    SampleSet *raw = nullptr;
    if (best >= 0) {
      raw = pool[best].release();
      pool.erase(pool.begin() + best);
    } else {
      const size_t bytes = need_x + need_i + 512;
      while (set_bytes + bytes > set_cap && !pool.empty()) {
        auto big = std::max_element(pool.begin(), pool.end(), [](const auto &a, const auto &b) {
          return a->x.cap + a->ids.cap < b->x.cap + b->ids.cap;
        });
        set_bytes -= (*big)->x.cap + (*big)->ids.cap;
        pool.erase(big);
      }
      if (set_bytes + bytes > set_cap) return nullptr;
      auto fresh = std::make_unique<SampleSet>();
      if (!fresh->x.ensure(need_x) || !fresh->ids.ensure(need_i)) return nullptr;
      set_bytes += fresh->x.cap + fresh->ids.cap;
      raw = fresh.release();
    }
    return std::shared_ptr<SampleSet>(raw, [this](SampleSet *q) { pool.emplace_back(q); });
  }

  // One-node sample reduction (Section 4.2 with the node's own lower bound
  // as beta): the samples it deletes are redundant in every descendant, so
  // the node's children and their subtrees are bounded over the samples it
  // keeps. Tried only when it can pay: the node's samples number at least
  // node_sr, some box has a half-diagonal shorter than sqrt(lb) (otherwise
  // every point lies at least that far from a corner of every box, and no
  // sample is redundant for the lower bound), and no box already holds more
  // than 3/4 of the samples as center candidates. A
  // result is kept when it deletes at least a quarter of the node's samples
  // and fits the memory cap; a try that deletes less makes the subtree wait
  // 1, 2, 4, ... generations before the next, a kept one 3.
  kc_status node_reduce(Node *m, const uint32_t *nin) {
    const kc_points p = pts_of(m);
    if (o.node_sr <= 0 || p.n < o.node_sr || !(m->lb > 0)) return KC_OK;
    if (m->sr_wait > 0) return KC_OK;
    bool small = false;
    uint32_t most = 0;
    for (int k = 0; k < K; ++k) {
      double r2 = 0;
      for (int a = 0; a < D; ++a) {
        const double hw = 0.5 * ((double)m->hi[k * D + a] - m->lo[k * D + a]);
        r2 += hw * hw;
      }
      if (r2 < m->lb) small = true;
      most = std::max(most, nin[k]);
    }
    if (!small || (double)most > 0.75 * (double)p.n) return KC_OK;
    in.reset();
    out.reset();
    std::vector<const std::vector<float> *> los{&m->lo}, his{&m->hi};
    std::vector<const Node *> ns{m};
    const BoxPlan P = plan_boxes(los, o.use_bt ? &ns : nullptr);
    const size_t o_n = out.take(8);
    kc_status s = reserve();
    if (s) return s;
    fill_boxes(P, los, his, o.use_bt ? &ns : nullptr);
    if ((s = upload())) return s;
    // count first; only a result worth keeping is compacted, straight into
    // buffers of its own size
    const kc_nodes nd = dev_nodes(P);
    const kc_refs rf = dev_refs(P);
    s = kc_reduce_count(h, &p, &nd, P.refs ? &rf : nullptr, m->lb, alpha_ub, out.dp<int64_t>(o_n), st);
    if (s) return s;
    res->passes++;
    res->node_sr_tries++;
    const double tq = now_s();
    if ((s = download("node reduction"))) return s;
    const int64_t n_out = *out.hp<int64_t>(o_n);
    if (o.verbose > 1)
      fprintf(stderr, "[node_sr] depth %d n %lld kept %lld lb/alpha %.3f wait %.3f ms\n", m->depth,
              (long long)p.n, (long long)n_out, m->lb / alpha_ub, (now_s() - tq) * 1e3);
    if (n_out < 1 || (double)n_out > 0.75 * (double)p.n) {
      // children skip 1, 2, 4, ... generations (sr_wait counts down per level)
      m->sr_backoff = (uint8_t)std::min(m->sr_backoff + 1, 6);
      m->sr_wait = (uint8_t)((1u << (m->sr_backoff - 1)) + 1);
      return KC_OK;
    }
    const int64_t ld = (n_out + 63) / 64 * 64;
    std::shared_ptr<SampleSet> S = take_set(ld);
    if (!S) return KC_OK;  // over the memory cap
    if ((s = kc_reduce_compact(h, &p, idx_of(m), n_out, S->x.as<float>(), S->ids.as<uint32_t>(), ld, st)))
      return s;
    S->n = n_out;
    S->ld = ld;
    m->ss = std::move(S);
    // the next three generations (bounds and boxes close to this node's)
    // keep the set as it is
    m->sr_backoff = 0;
    m->sr_wait = 4;
    res->node_sr_kept++;
    return KC_OK;
  }

  // Morton order of the active samples over the root box (the kernels'
  // results do not depend on the order; coherent wavefronts make them faster).
  kc_status spatial_order() {
    const int nxt = cur == 0 ? 1 : 0;
    if (!xbuf[nxt].ensure((size_t)D * X0->ld * 4) || !ibuf[nxt].ensure((size_t)X0->ld * 4))
      return kc_fail(h, KC_ENOMEM, "sample buffers");
    kc_status s = kc_spatial_order(h, &act, idx, root_lo.data(), root_hi.data(), xbuf[nxt].as<float>(),
                                   ibuf[nxt].as<uint32_t>(), X0->ld, st);
    if (s) return s;
    cur = nxt;
    act.x = xbuf[cur].as<float>();
    act.ld = X0->ld;
    idx = ibuf[cur].as<uint32_t>();
    return KC_OK;
  }

  // ------------------------------------------------------------ features --
  // 32 features of candidate (k,a) of node m (tightened boxes), see the
  // branching network's documentation.
  void features(const Node *m, int bi, int nbatch, const uint32_t *nin, const uint32_t *nasg,
                int k, int a, float *f) const {
    const double al = alpha_ub > 0 ? alpha_ub : 1.0;
    const double glb = global_lb();
    double wmax = 0.0;
    for (int q = 0; q < K * D; ++q) wmax = std::max(wmax, (double)m->hi[q] - m->lo[q]);
    const double w = (double)m->hi[k * D + a] - m->lo[k * D + a];
    const double rw = std::max(1e-30, (double)root_hi[a] - root_lo[a]);
    int rank = 0;
    for (int q = 0; q < K * D; ++q)
      if ((double)m->hi[q] - m->lo[q] > w) ++rank;
    double logvol = 0.0;
    for (int b = 0; b < D; ++b) {
      const double rb = std::max(1e-30, (double)root_hi[b] - root_lo[b]);
      logvol += std::log(((double)m->hi[k * D + b] - m->lo[k * D + b]) / rb + 1e-12);
    }
    // distance of the LB sample to every box
    int nearest = 0;
    double dk = 0.0, dbest = INFINITY;
    for (int kk = 0; kk < K; ++kk) {
      double s = 0;
      for (int b = 0; b < D; ++b) {
        const double x = m->xstar[b];
        const double c = std::min(std::max(x, (double)m->lo[kk * D + b]), (double)m->hi[kk * D + b]);
        s += (x - c) * (x - c);
      }
      if (s < dbest) {
        dbest = s;
        nearest = kk;
      }
      if (kk == k) dk = s;
    }
    const double lo = m->lo[k * D + a], hi = m->hi[k * D + a];
    const double xs = m->xstar[a];
    double pos = w > 0 ? (xs - lo) / w : 0.5;
    pos = std::min(2.0, std::max(-1.0, pos));
    double overlap = 0.0, mind = INFINITY;
    for (int kk = 0; kk < K; ++kk) {
      if (kk == k) continue;
      const double l2 = m->lo[kk * D + a], h2 = m->hi[kk * D + a];
      overlap += std::max(0.0, std::min(hi, h2) - std::max(lo, l2));
      double s = 0;
      for (int b = 0; b < D; ++b) {
        const double c1 = 0.5 * ((double)m->lo[k * D + b] + m->hi[k * D + b]);
        const double c2 = 0.5 * ((double)m->lo[kk * D + b] + m->hi[kk * D + b]);
        s += (c1 - c2) * (c1 - c2);
      }
      mind = std::min(mind, std::sqrt(s));
    }
    const double nact = (double)(m->ss ? m->ss->n : act.n), n0 = (double)X0->n;
    const int q = k * D + a;
    const double mean_l = pc_cnt[0][q] ? pc_sum[0][q] / pc_cnt[0][q] : 0.0;
    const double mean_r = pc_cnt[1][q] ? pc_sum[1][q] / pc_cnt[1][q] : 0.0;
    int nref = 0;
    if (!m->roff.empty())
      for (int kk = 0; kk < K; ++kk) nref += m->roff[kk + 1] > m->roff[kk];
    f[0] = (float)(m->depth / 32.0);
    f[1] = (float)(std::log1p((double)heap.size()) / 10.0);
    f[2] = (float)std::min(2.0, m->lb / al);
    f[3] = (float)std::max(-1.0, (alpha_ub - m->lb) / al);
    f[4] = (float)std::max(-1.0, (alpha_ub - glb) / al);
    f[5] = (float)((m->lb - m->parent_lb) / al);
    f[6] = (float)(K / 16.0);
    f[7] = (float)(D / 16.0);
    f[8] = (float)(nact / n0);
    f[9] = seeds ? 1.f : 0.f;
    f[10] = (float)((double)nref / K);
    f[11] = (float)((double)bi / std::max(1, nbatch));
    f[12] = (float)(w / rw);
    f[13] = (float)(wmax > 0 ? w / wmax : 0.0);
    f[14] = (float)((double)rank / (K * D));
    f[15] = (float)(logvol / D / 10.0);
    f[16] = (float)(std::log1p((double)nin[k]) / std::log1p(n0));
    f[17] = (float)(std::log1p((double)nasg[k]) / std::log1p(n0));
    f[18] = nearest == k ? 1.f : 0.f;
    f[19] = (float)std::min(4.0, dk / al);
    f[20] = (float)pos;
    f[21] = (xs < lo || xs > hi) ? 1.f : 0.f;
    f[22] = (float)((0.5 * (lo + hi) - root_lo[a]) / rw);
    f[23] = (float)(w > 0 ? std::min(8.0, overlap / w) : 0.0);
    f[24] = (float)(std::isfinite(mind) ? std::min(8.0, mind / std::sqrt(al)) : 8.0);
    f[25] = (float)((double)m->nsplit[q] / (m->depth + 1));
    f[26] = (float)std::max(-1.0, std::min(4.0, mean_l));
    f[27] = (float)std::max(-1.0, std::min(4.0, mean_r));
    f[28] = (float)(std::log1p((double)pc_cnt[0][q]) / 10.0);
    f[29] = (float)(std::log1p((double)pc_cnt[1][q]) / 10.0);
    f[30] = (float)((0.5 * (lo + hi) - root_lo[a]) / rw - 0.5);
    f[31] = 0.f;
  }

  // Picks (k,a) for every node to branch. Max-range rule (Section 3.3):
  // widest box side, lowest k then a on ties; learned rule: highest network
  // score among positive-width candidates, max-range when the network is off.
  kc_status choose(const std::vector<Node *> &nodes, const std::vector<int> &bidx,
                   std::vector<int> &ck, std::vector<int> &ca) {
    const int nn = (int)nodes.size();
    ck.assign(nn, -1);
    ca.assign(nn, -1);
    for (int i = 0; i < nn; ++i) {
      const Node *m = nodes[i];
      double bw = 0.0;
      for (int k = 0; k < K; ++k)
        for (int a = 0; a < D; ++a) {
          const double w = (double)m->hi[k * D + a] - m->lo[k * D + a];
          if (w > bw) {
            bw = w;
            ck[i] = k;
            ca[i] = a;
          }
        }
    }
    if (o.branching != 1 || !o.mlp_w) return KC_OK;
    std::vector<int> row_node, row_q;
    for (int i = 0; i < nn; ++i) {
      const Node *m = nodes[i];
      const double wmax = max_width(m);
      for (int q = 0; q < K * D; ++q) {
        const double w = (double)m->hi[q] - m->lo[q];
        if (w > 0 && w >= kWideFrac * wmax) {
          row_node.push_back(i);
          row_q.push_back(q);
        }
      }
    }
    const int64_t rows = (int64_t)row_node.size();
    if (rows == 0) return KC_OK;
    in.reset();
    out.reset();
    const size_t o_f = in.take((size_t)rows * NFEAT * 4);
    const size_t o_s = out.take((size_t)rows * 4);
    kc_status s = reserve();
    if (s) return s;
    float *feat = in.hp<float>(o_f);
    for (int64_t r = 0; r < rows; ++r) {
      const int i = row_node[r];
      features(nodes[i], bidx[i], nn, &ta.nin[(size_t)bidx[i] * K], &ta.nasg[(size_t)bidx[i] * K],
               row_q[r] / D, row_q[r] % D, feat + r * NFEAT);
    }
    if ((s = upload())) return s;
    s = kc_mlp_forward(h, o.mlp_w, in.dp<float>(o_f), rows, out.dp<float>(o_s), nullptr, st);
    if (s) return s;
    if ((s = download("branching network"))) return s;
    const float *sc = out.hp<float>(o_s);
    std::vector<float> best(nn, -INFINITY);
    for (int64_t r = 0; r < rows; ++r) {
      const int i = row_node[r];
      if (sc[r] > best[i]) {  // first (lowest (k,a)) wins ties
        best[i] = sc[r];
        ck[i] = row_q[r] / D;
        ca[i] = row_q[r] % D;
      }
    }
    return KC_OK;
  }

  // Strong branching at labelled nodes: every positive-width (k,a) is split,
  // both children bounded in one launch; score = max(dL, e) * max(dR, e).
  kc_status strong_branching(const std::vector<Node *> &nodes, const std::vector<int> &bidx) {
    std::vector<std::vector<float>> clo, chi;
    struct Cand {
      int node, k, a;
    };
    std::vector<Cand> cands;
    for (int i = 0; i < (int)nodes.size(); ++i) {
      const Node *m = nodes[i];
      const double wmax = max_width(m);
      for (int k = 0; k < K; ++k)
        for (int a = 0; a < D; ++a) {
          const float l = m->lo[k * D + a], hh = m->hi[k * D + a];
          if (!(l < hh) || (double)hh - l < kWideFrac * wmax) continue;
          float lh, rl;
          split_interval(l, hh, &lh, &rl);
          std::vector<float> L1 = m->lo, H1 = m->hi, L2 = m->lo, H2 = m->hi;
          H1[k * D + a] = lh;
          L2[k * D + a] = rl;
          clo.push_back(L1);
          chi.push_back(H1);
          clo.push_back(L2);
          chi.push_back(H2);
          cands.push_back({i, k, a});
        }
    }
    if (cands.empty()) return KC_OK;
    // children of nodes sharing their samples form one launch (cands are in
    // node order, two children each)
    std::vector<std::pair<int, int>> R;  // child ranges
    std::vector<const Node *> rn;        // a node of each range
    for (size_t c = 0; c < cands.size();) {
      size_t e = c + 1;
      while (e < cands.size() && nodes[cands[e].node]->ss == nodes[cands[c].node]->ss) ++e;
      R.push_back({(int)(2 * c), (int)(2 * e)});
      rn.push_back(nodes[cands[c].node]);
      c = e;
    }
    const int ne = (int)clo.size();
    in.reset();
    out.reset();
    std::vector<BoxPlan> plans;
    std::vector<std::vector<const std::vector<float> *>> glo(R.size()), ghi(R.size());
    for (size_t g = 0; g < R.size(); ++g) {
      for (int j = R[g].first; j < R[g].second; ++j) {
        glo[g].push_back(&clo[j]);
        ghi[g].push_back(&chi[j]);
      }
      plans.push_back(plan_boxes(glo[g], nullptr));
    }
    const size_t o_lb = out.take((size_t)ne * 8), o_c = out.take((size_t)ne * K * 8);
    kc_status s = reserve();
    if (s) return s;
    for (size_t g = 0; g < R.size(); ++g) fill_boxes(plans[g], glo[g], ghi[g], nullptr);
    if ((s = upload())) return s;
    for (size_t g = 0; g < R.size(); ++g) {
      const size_t j0 = (size_t)R[g].first;
      const kc_points p = pts_of(rn[g]);
      const kc_nodes nd = dev_nodes(plans[g]);
      s = kc_lower_bound(h, &p, &nd, nullptr, out.dp<double>(o_lb) + j0, nullptr,
                         out.dp<int64_t>(o_c) + j0 * K, st);
      if (s) return s;
    }
    if ((s = download("strong branching"))) return s;
    const double *lb = out.hp<double>(o_lb);
    const int64_t *cand = out.hp<int64_t>(o_c);
    const double al = alpha_ub;
    const double e = 1e-6 * al;
    int last = -1;
    for (size_t c = 0; c < cands.size(); ++c) {
      const Node *m = nodes[cands[c].node];
      double g[2];
      for (int side = 0; side < 2; ++side) {
        const int j = (int)(2 * c + side);
        bool empty = false;
        for (int k = 0; k < K; ++k)
          if (cand[(size_t)j * K + k] < 0) empty = true;
        const double clb = empty ? al : std::min(al, std::max(m->lb, lb[j]));
        g[side] = std::max(clb - m->lb, e);
      }
      if (sb_rows >= o.sb_cap) break;
      if (cands[c].node != last) {
        last = cands[c].node;
        ++sb_nodes;
      }
      features(m, bidx[cands[c].node], (int)nodes.size(), &ta.nin[(size_t)bidx[cands[c].node] * K],
               &ta.nasg[(size_t)bidx[cands[c].node] * K], cands[c].k, cands[c].a,
               &o.sb_feat[(size_t)sb_rows * NFEAT]);
      o.sb_score[sb_rows] = (float)(g[0] * g[1] / (al * al));
      o.sb_node[sb_rows] = sb_nodes - 1;
      if (o.sb_lo && o.sb_hi) {
        std::memcpy(o.sb_lo + (size_t)sb_rows * K * D, m->lo.data(), (size_t)K * D * 4);
        std::memcpy(o.sb_hi + (size_t)sb_rows * K * D, m->hi.data(), (size_t)K * D * 4);
      }
      if (o.sb_ka) {
        o.sb_ka[2 * sb_rows] = cands[c].k;
        o.sb_ka[2 * sb_rows + 1] = cands[c].a;
      }
      if (o.sb_bounds) {
        o.sb_bounds[2 * sb_rows] = m->lb;
        o.sb_bounds[2 * sb_rows + 1] = al;
      }
      ++sb_rows;
    }
    return KC_OK;
  }

  // --------------------------------------------------------------- run --
  kc_status run() {
    t0 = now_s();
    if (hipStreamCreate(&st) != hipSuccess) return kc_fail(h, KC_EDEVICE, "stream");
    kc_status s = root();
    if (s) return s;
    if (!o.keep_order && act.n >= (1 << 16) && (s = spatial_order())) return s;
    if (o.node_sr > 0) {
      // subtree sets may hold up to half of the memory free now
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) != hipSuccess) return kc_fail(h, KC_EDEVICE, "memory info");
      set_cap = fr / 2;
    }
    int64_t passes_since_sr = 0;
    res->status = 0;
    std::vector<Node *> batch;
    std::vector<char> alive;
    while (!heap.empty()) {
      if (o.max_nodes > 0 && res->nodes >= o.max_nodes) {
        res->status = 1;
        break;
      }
      if (o.time_limit_s > 0 && now_s() - t0 > o.time_limit_s) {
        res->status = 2;
        break;
      }
      // node selection: least lower bound first
      batch.clear();
      const double thr = prune_thr();
      while ((int)batch.size() < o.batch && !heap.empty()) {
        Node *m = heap_pop();
        if (m->lb >= thr) {
          lb_closed = std::min(lb_closed, m->lb);
          delete m;
          continue;
        }
        batch.push_back(m);
      }
      if (batch.empty()) break;
      res->nodes += (int64_t)batch.size();
      {
        const std::vector<int> perm = group_order(batch);
        std::vector<Node *> b2(batch.size());
        for (size_t i = 0; i < perm.size(); ++i) b2[i] = batch[perm[i]];
        batch.swap(b2);
      }

      // bounds tightening
      const double a_bt = o.use_bt ? alpha_ub : INFINITY;
      double tp = now_s();
      const int64_t evals_start = res->evals + res->tighten_evals;
      if ((s = tighten(batch, alive, a_bt))) return s;
      t_tighten += now_s() - tp;
      std::vector<Node *> live;
      std::vector<int> bidx;
      for (size_t i = 0; i < batch.size(); ++i) {
        if (alive[i]) {
          live.push_back(batch[i]);
          bidx.push_back((int)i);
        } else {
          lb_closed = std::min(lb_closed, std::max(batch[i]->lb, a_bt));
          delete batch[i];
        }
      }
      // sample reduction every i_sr passes, over the open nodes and this
      // batch, when it can delete anything (can_reduce); otherwise it is
      // tried again at the next pass. A reduction that deletes under 1% of
      // the active samples doubles the interval (up to 64 i_sr), any other
      // resets it to i_sr. The rules count samples and box sizes, not time,
      // so the schedule of a solve does not depend on kernel speed.
      ++passes_since_sr;
      if (o.i_sr > 0 && sr_interval == 0) sr_interval = o.i_sr;
      if (o.i_sr > 0 && passes_since_sr >= sr_interval && can_reduce(live)) {
        passes_since_sr = 0;
        tp = now_s();
        const int64_t before = act.n;
        int64_t kept = before;
        if ((s = reduce(live, &kept))) return s;
        ++sr_runs;
        const double cost = now_s() - tp;
        if ((double)(before - kept) < 0.01 * (double)before)
          sr_interval = std::min<int64_t>(sr_interval * 2, (int64_t)o.i_sr * 64);
        else
          sr_interval = o.i_sr;
        t_reduce += cost;
      }
      tp = now_s();

      // branching; a node whose boxes are all single points is a leaf
      std::vector<Node *> to_branch, leaves;
      std::vector<int> to_branch_bidx;
      for (size_t i = 0; i < live.size(); ++i) {
        Node *m = live[i];
        bool leaf = true;
        for (int q = 0; q < K * D; ++q)
          if (m->lo[q] != m->hi[q]) leaf = false;
        if (leaf)
          leaves.push_back(m);
        else {
          to_branch.push_back(m);
          to_branch_bidx.push_back(bidx[i]);
        }
      }
      // one-node reductions give subtrees their own samples. A try over n
      // samples is priced at 2 K n sample-box evaluations (redundancy tests
      // of K boxes, scan, read-back); the tries of a pass stay within a
      // quarter of the previous pass's evaluations, and a node is tried only
      // while at least a quarter of the recent tries at its lb / alpha (in
      // tenths) were kept. One try every 16 passes goes ahead regardless, so
      // the rates can recover. These rules count work, not time.
      ++n_pass;
      if (o.node_sr > 0) {
        const double tn = now_s();
        double budget = 0.25 * (double)last_pass_evals;
        bool force = n_pass - nsr_last_pass >= 16;
        for (size_t i = 0; i < to_branch.size(); ++i) {
          Node *m = to_branch[i];
          const double cost = 2.0 * K * (double)pts_of(m).n;
          const int bk = std::max(0, std::min(9, (int)(10.0 * m->lb / alpha_ub)));
          if ((cost > budget || nsr_keep_rate[bk] < 0.25) && !force) continue;
          const int64_t tries = res->node_sr_tries, kept = res->node_sr_kept;
          if ((s = node_reduce(m, &ta.nin[(size_t)to_branch_bidx[i] * K]))) return s;
          if (res->node_sr_tries > tries) {
            nsr_keep_rate[bk] = 0.9 * nsr_keep_rate[bk] + (res->node_sr_kept > kept ? 0.1 : 0.0);
            budget -= cost;
            force = false;
            nsr_last_pass = n_pass;
          }
        }
        t_reduce += now_s() - tn;
        tp += now_s() - tn;
      }
      std::vector<int> ck, ca;
      if ((s = choose(to_branch, to_branch_bidx, ck, ca))) return s;
      if (o.sb_every > 0 && o.sb_feat && o.sb_score && o.sb_node) {
        std::vector<Node *> lab;
        std::vector<int> lab_b;
        for (size_t i = 0; i < to_branch.size(); ++i) {
          const int64_t ord = n_branched + (int64_t)i;
          if (ord < o.sb_first || (ord - o.sb_first) % o.sb_every == 0) {
            lab.push_back(to_branch[i]);
            lab_b.push_back(to_branch_bidx[i]);
          }
        }
        if (!lab.empty() && sb_rows < o.sb_cap)
          if ((s = strong_branching(lab, lab_b))) return s;
      }
      n_branched += (int64_t)to_branch.size();

      // children (and leaves) to bound
      std::vector<Node *> ev;
      std::vector<char> is_leaf;
      for (size_t i = 0; i < to_branch.size(); ++i) {
        Node *m = to_branch[i];
        const int k = ck[i], a = ca[i];
        float lh, rl;
        split_interval(m->lo[k * D + a], m->hi[k * D + a], &lh, &rl);
        for (int side = 0; side < 2; ++side) {
          Node *c = new Node();
          c->lo = m->lo;
          c->hi = m->hi;
          if (side == 0)
            c->hi[k * D + a] = lh;
          else
            c->lo[k * D + a] = rl;
          c->parent_lb = m->lb;
          c->lb = m->lb;
          c->depth = m->depth + 1;
          c->split_k = k;
          c->split_a = a;
          c->side = side;
          c->nsplit = m->nsplit;
          if (c->nsplit[k * D + a] < 255) c->nsplit[k * D + a]++;
          inherit_refs(m, c);
          c->ss = m->ss;
          c->sr_backoff = m->sr_backoff;
          c->sr_wait = m->sr_wait > 0 ? (uint8_t)(m->sr_wait - 1) : 0;
          c->id = next_id++;
          if (symmetry && !apply_symmetry(c->lo, c->hi)) {
            delete c;  // empty box: no solution
            continue;
          }
          ev.push_back(c);
          is_leaf.push_back(0);
        }
        delete m;
      }
      for (Node *m : leaves) {
        ev.push_back(m);
        is_leaf.push_back(1);
      }
      t_branch += now_s() - tp;
      tp = now_s();
      if (!ev.empty())
        if ((s = bound(ev, is_leaf))) return s;
      t_bound += now_s() - tp;
      last_pass_evals = res->evals + res->tighten_evals - evals_start;

      if (!heap.empty()) {
        const double lb = global_lb();
        // alpha_ub bounds the best set's objective from above, so the gap
        // after its certificate is no larger
        if (alpha_ub - lb <= o.eps_rel * alpha_ub) break;
      }
      if (o.verbose && (res->nodes % (o.batch * 20) < o.batch))
        fprintf(stderr,
                "[kc_solve] nodes %lld open %zu n_active %lld subtree sets %.3f GB alpha %.9g lb %.9g "
                "t %.2fs\n",
                (long long)res->nodes, heap.size(), (long long)act.n, set_bytes * 1e-9, alpha_ub,
                global_lb(), now_s() - t0);
    }
    if (o.verbose)
      fprintf(stderr,
              "[kc_solve] phases: tighten %.3fs reduce %.3fs (%lld runs) branch %.3fs bound %.3fs "
              "total %.3fs; bounded %lld nodes, %lld pruned by their bound\n",
              t_tighten, t_reduce, (long long)sr_runs, t_branch, t_bound, now_s() - t0,
              (long long)n_bounded, (long long)n_bounded_pruned);
    return KC_OK;
  }

  // Bounds every node of `ev`: lower bound + candidates in one launch, the
  // candidates' objective in one float32 launch (coordinates gathered on the
  // device), float64 certificate of an improvement. Children with an empty
  // box are dropped; leaves leave the tree.
  kc_status bound(std::vector<Node *> &ev_in, const std::vector<char> &leaf_in) {
    const int ne = (int)ev_in.size();
    // nodes sharing their samples next to each other: one launch per run
    std::vector<Node *> ev(ne);
    std::vector<char> is_leaf(ne);
    {
      const std::vector<int> perm = group_order(ev_in);
      for (int i = 0; i < ne; ++i) {
        ev[i] = ev_in[perm[i]];
        is_leaf[i] = leaf_in[perm[i]];
      }
    }
    const auto R = runs(ev);
    in.reset();
    out.reset();
    std::vector<BoxPlan> plans;
    std::vector<std::vector<const std::vector<float> *>> glo(R.size()), ghi(R.size());
    for (size_t g = 0; g < R.size(); ++g) {
      for (int i = R[g].first; i < R[g].second; ++i) {
        glo[g].push_back(&ev[i]->lo);
        ghi[g].push_back(&ev[i]->hi);
      }
      plans.push_back(plan_boxes(glo[g], nullptr));
    }
    const size_t ng = (size_t)ne * K + ne;  // candidates, then the LB samples
    const size_t o_lb = out.take((size_t)ne * 8), o_ids = out.take(ng * 8),
                 o_xy = out.take(ng * D * 4), o_orig = out.take(ng * 8),
                 o_obj = out.take((size_t)ne * 8), o_oam = out.take((size_t)ne * 8),
                 o_l64 = out.take((size_t)ne * 8);
    kc_status s = reserve();
    if (s) return s;
    for (size_t g = 0; g < R.size(); ++g) fill_boxes(plans[g], glo[g], ghi[g], nullptr);
    if ((s = upload())) return s;
    int64_t *ids = out.dp<int64_t>(o_ids);
    int64_t *orig = out.dp<int64_t>(o_orig);
    float *dxy = out.dp<float>(o_xy);
    if (o.autotune)  // shapes new to the handle's table: sweep the tiles first
      for (size_t g = 0; g < R.size(); ++g) {
        const kc_points p = pts_of(ev[R[g].first]);
        const kc_nodes nd = dev_nodes(plans[g]);
        if (!kc_bound_tuned(h, &p, &nd, true) && (s = kc_autotune(h, &p, &nd, 1, nullptr, st)))
          return s;
      }
    (void)hipEventRecord(h->ev0, st);
    for (size_t g = 0; g < R.size(); ++g) {
      const size_t i0 = (size_t)R[g].first, gn = (size_t)(R[g].second - R[g].first);
      const kc_points p = pts_of(ev[i0]);
      const kc_nodes nd = dev_nodes(plans[g]);
      s = kc_lower_bound(h, &p, &nd, nullptr, out.dp<double>(o_lb) + i0, ids + (size_t)ne * K + i0,
                         ids + i0 * K, st);
      if (s) return s;
      res->passes++;
      res->evals += p.n * (int64_t)gn * K;
    }
    (void)hipEventRecord(h->ev1, st);
    for (size_t g = 0; g < R.size(); ++g) {
      const size_t i0 = (size_t)R[g].first, gn = (size_t)(R[g].second - R[g].first);
      const kc_points p = pts_of(ev[i0]);
      const uint32_t *ix = idx_of(ev[i0]);
      if ((s = kc_gather(h, &p, ids + i0 * K, (int)(gn * K), ix, dxy + i0 * K * D, orig + i0 * K, st)))
        return s;
      if ((s = kc_gather(h, &p, ids + (size_t)ne * K + i0, (int)gn, ix, dxy + ((size_t)ne * K + i0) * D,
                         orig + (size_t)ne * K + i0, st)))
        return s;
      if (o.autotune) {  // a shape new to the handle's table: sweep the tiles first
        bool tuned = false;
        (void)kc_objective_tile(h, &p, (int)gn, K, &tuned);
        if (!tuned && (s = kc_autotune_objective(h, &p, (int)gn, K, dxy + i0 * K * D, st)))
          return s;
      }
    }
    // the objective of every candidate set (a set with an empty box reads
    // sample 0 in its place; its value is never used); over the node's
    // samples it equals the objective over all samples, since a deleted
    // sample lies closer than the node's bound to any centers in its boxes
    (void)hipEventRecord(h->ev2, st);
    for (size_t g = 0; g < R.size(); ++g) {
      const size_t i0 = (size_t)R[g].first, gn = (size_t)(R[g].second - R[g].first);
      const kc_points p = pts_of(ev[i0]);
      // each set's centers lie in its node's boxes, so the node's lower
      // bound is a lower bound of the set's objective; the node's lower-bound
      // sample (farthest from its boxes) is the set's witness
      s = kc_objective_screen_witness(h, &p, (int)gn, K, dxy + i0 * K * D, screen_cut(),
                                      out.dp<double>(o_lb) + i0, dxy + ((size_t)ne * K + i0) * D,
                                      ids + (size_t)ne * K + i0, out.dp<double>(o_obj) + i0,
                                      out.dp<int64_t>(o_oam) + i0, st);
      if (s) return s;
      res->passes++;
      res->obj_evals += p.n * (int64_t)gn * K;
    }
    (void)hipEventRecord(h->ev3, st);
    if ((s = download("bound"))) return s;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, h->ev0, h->ev1);
    res->lb_kernel_ms += ms;
    (void)hipEventElapsedTime(&ms, h->ev2, h->ev3);
    res->obj_kernel_ms += ms;
    const double *lb = out.hp<double>(o_lb);
    const int64_t *cand = out.hp<int64_t>(o_ids);
    const float *xy = out.hp<float>(o_xy);
    const int64_t *horig = out.hp<int64_t>(o_orig);
    const double *ub = out.hp<double>(o_obj);

    std::vector<char> ok(ne, 1);
    int best = -1;
    for (int i = 0; i < ne; ++i) {
      for (int k = 0; k < K; ++k)
        if (cand[(size_t)i * K + k] < 0) ok[i] = 0;  // no sample in some box
      if (ok[i] && ub[i] < alpha_ub && (best < 0 || ub[i] < ub[best])) best = i;
    }
    if (best >= 0) {  // the new incumbent bound; certified when the search ends
      alpha_ub = ub[best];
      pending = true;
      pend_ids.assign(horig + (size_t)best * K, horig + (size_t)best * K + K);
      pend_coords.assign(xy + (size_t)best * K * D, xy + (size_t)best * K * D + K * D);
    }
    const double thr = prune_thr();
    const double rel = kc_rel_margin(D) + 0x1p-50, eta = kc_abs_margin(D);
    for (int i = 0; i < ne; ++i) {
      ++n_bounded;
      if (!is_leaf[i] && std::max(ev[i]->lb, lb[i]) >= thr) ++n_bounded_pruned;
    }
    // A leaf's only solution is its single-point centers. The float32 screen
    // bounds their objective from below by ub (1 - 2 gamma) only, which at
    // many attributes lies more than eps_rel below the incumbent when the leaf
    // ties it; such leaves get their objective in float64 (over the leaf's
    // samples, which give the objective over all samples), so that the final
    // gap closes.
    std::vector<double> leaf64(ne, -1.0);
    {
      std::vector<int> band;
      for (int i = 0; i < ne; ++i) {
        if (!is_leaf[i] || !ok[i]) continue;
        const double lo_obj = std::max(0.0, (ub[i] - eta) / (1.0 + rel) * (1.0 - rel) - eta);
        if (std::max(ev[i]->lb, lo_obj) < alpha_ub * (1.0 - o.eps_rel)) band.push_back(i);
      }
      if (!band.empty()) {
        double *d64 = out.dp<double>(o_l64), *h64 = out.hp<double>(o_l64);
        for (const int i : band) {
          const kc_points p = pts_of(ev[i]);
          if ((s = kc_objective(h, &p, 1, K, out.dp<float>(o_xy) + (size_t)i * K * D, 64, d64 + i,
                                nullptr, st)))
            return s;
          res->passes++;
        }
        if (hipMemcpyAsync(h64, d64, (size_t)ne * 8, hipMemcpyDeviceToHost, st) != hipSuccess)
          return kc_fail(h, KC_EDEVICE, "download");
        if ((s = sync("leaf certificate"))) return s;
        for (const int i : band) leaf64[i] = h64[i];
      }
    }
    for (int i = 0; i < ne; ++i) {
      Node *m = ev[i];
      if (!ok[i]) {
        delete m;  // the node holds no feasible centers
        continue;
      }
      m->lb = std::max(m->lb, lb[i]);
      std::memcpy(m->xstar, xy + ((size_t)ne * K + i) * D, (size_t)D * 4);
      if (!is_leaf[i] && m->split_k >= 0) {
        const int q = m->split_k * D + m->split_a;
        pc_sum[m->side][q] += (m->lb - m->parent_lb) / (alpha_ub > 0 ? alpha_ub : 1.0);
        pc_cnt[m->side][q]++;
      }
      if (is_leaf[i]) {
        // every box is one point: the node's only solution has objective ub[i]
        // (float32, rounded up), or leaf64[i] (float64, within (D+3) 2^-53)
        double lo_obj = std::max(0.0, (ub[i] - eta) / (1.0 + rel) * (1.0 - rel) - eta);
        if (leaf64[i] >= 0.0) lo_obj = std::max(lo_obj, leaf64[i] * (1.0 - (D + 3) * 0x1p-52));
        lb_closed = std::min(lb_closed, std::max(m->lb, lo_obj));
        delete m;
      } else if (m->lb >= thr) {
        lb_closed = std::min(lb_closed, m->lb);
        delete m;
      } else {
        heap_push(m);
      }
    }
    return KC_OK;
  }
};

}  // namespace

extern "C" kc_status kc_solve(kc_handle *h, const kc_points *pts, const kc_opts *opts,
                              kc_result *res) {
  return kc_guard(h, [&]() -> kc_status {
    if (!h) return KC_EINVAL;
    kc_status s = kc_validate_points(h, pts);
    if (s != KC_OK) return s;
    KC_RETURN_IF(!opts || !res, h, KC_EINVAL, "opts / result is NULL");
    KC_RETURN_IF(opts->k < 1 || opts->k > 64 || opts->k > pts->n, h, KC_EINVAL,
                 "k must be in [1, min(64, n)] (got %d)", opts->k);
    KC_RETURN_IF(opts->batch < 1, h, KC_EINVAL, "batch must be >= 1");
    KC_RETURN_IF(opts->fft_start < 0 || opts->fft_start >= pts->n, h, KC_EINVAL,
                 "fft_start out of range");
    KC_RETURN_IF(!(opts->eps_rel >= 0.0 && opts->eps_rel < 1.0), h, KC_EINVAL, "eps_rel in [0,1)");
    KC_RETURN_IF(opts->max_refs < 0 || opts->max_refs > 64, h, KC_EINVAL, "max_refs in [0,64]");
    KC_RETURN_IF(opts->node_sr < 0, h, KC_EINVAL, "node_sr must be >= 0");
    KC_RETURN_IF(opts->branching == 1 && !opts->mlp_w, h, KC_EINVAL, "learned branching needs mlp_w");
    KC_RETURN_IF(opts->sb_every > 0 && (!opts->sb_feat || !opts->sb_score || !opts->sb_node || opts->sb_cap < 1),
                 h, KC_EINVAL, "strong-branching labels need their host arrays");
    std::memset(res, 0, sizeof(*res));
    Solver S(h, pts, opts, res);
    const double t0 = now_s();
    s = S.run();
    if (s == KC_OK) s = S.certify();
    if (s != KC_OK) {
      (void)hipDeviceSynchronize();
      return s;
    }
    res->obj = S.alpha_cert;
    res->lb = S.global_lb();
    res->gap = S.alpha_cert > 0 ? (S.alpha_cert - res->lb) / S.alpha_cert : 0.0;
    // the open set ran out, but the certified gap is above eps_rel
    if (res->status == 0 && res->gap > opts->eps_rel) res->status = 3;
    for (int k = 0; k < opts->k; ++k) res->centers[k] = S.inc_ids[k];
    res->n_active = S.act.n;
    res->sb_rows = S.sb_rows;
    res->sb_nodes = S.sb_nodes;
    res->seconds = now_s() - t0;
    return KC_OK;
  });
}
