// kc_bound.hip -- kc_lower_bound / kc_objective entry points, launch sizing
// and the kernels that reduce the per-split partial results.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>

#include "kc_bound_impl.h"

namespace kcb {
kc_status launch_d0(int, int, int, bool, int, const BoundArgs &, int, size_t, hipStream_t);
kc_status launch_d1(int, int, int, bool, int, const BoundArgs &, int, size_t, hipStream_t);
kc_status launch_d2(int, int, int, bool, int, const BoundArgs &, int, size_t, hipStream_t);
kc_status launch_d3(int, int, int, bool, int, const BoundArgs &, int, size_t, hipStream_t);
kc_status launch_d4(int, int, int, bool, int, const BoundArgs &, int, size_t, hipStream_t);
kc_status launch_d5(int, int, int, bool, int, const BoundArgs &, int, size_t, hipStream_t);
kc_status launch_d6(int, int, int, bool, int, const BoundArgs &, int, size_t, hipStream_t);
kc_status launch_d7(int, int, int, bool, int, const BoundArgs &, int, size_t, hipStream_t);
kc_status launch_d8(int, int, int, bool, int, const BoundArgs &, int, size_t, hipStream_t);
kc_status launch_obj64_d0(const Obj64Args &, int, size_t, hipStream_t);
kc_status launch_obj64_d1(const Obj64Args &, int, size_t, hipStream_t);
kc_status launch_obj64_d2(const Obj64Args &, int, size_t, hipStream_t);
kc_status launch_obj64_d3(const Obj64Args &, int, size_t, hipStream_t);
kc_status launch_obj64_d4(const Obj64Args &, int, size_t, hipStream_t);
kc_status launch_obj64_d5(const Obj64Args &, int, size_t, hipStream_t);
kc_status launch_obj64_d6(const Obj64Args &, int, size_t, hipStream_t);
kc_status launch_obj64_d7(const Obj64Args &, int, size_t, hipStream_t);
kc_status launch_obj64_d8(const Obj64Args &, int, size_t, hipStream_t);

static kc_status dispatch(int d, int S, int NG, int KC, bool point, int skip, const BoundArgs &A,
                          int grid, size_t lds, hipStream_t st) {
  switch (d) {
    case 1: return launch_d1(S, NG, KC, point, skip, A, grid, lds, st);
    case 2: return launch_d2(S, NG, KC, point, skip, A, grid, lds, st);
    case 3: return launch_d3(S, NG, KC, point, skip, A, grid, lds, st);
    case 4: return launch_d4(S, NG, KC, point, skip, A, grid, lds, st);
    case 5: return launch_d5(S, NG, KC, point, skip, A, grid, lds, st);
    case 6: return launch_d6(S, NG, KC, point, skip, A, grid, lds, st);
    case 7: return launch_d7(S, NG, KC, point, skip, A, grid, lds, st);
    case 8: return launch_d8(S, NG, KC, point, skip, A, grid, lds, st);
    default: return launch_d0(S, NG, KC, point, skip, A, grid, lds, st);
  }
}

static kc_status dispatch64(int d, const Obj64Args &A, int splits, size_t lds, hipStream_t st) {
  switch (d) {
    case 1: return launch_obj64_d1(A, splits, lds, st);
    case 2: return launch_obj64_d2(A, splits, lds, st);
    case 3: return launch_obj64_d3(A, splits, lds, st);
    case 4: return launch_obj64_d4(A, splits, lds, st);
    case 5: return launch_obj64_d5(A, splits, lds, st);
    case 6: return launch_obj64_d6(A, splits, lds, st);
    case 7: return launch_obj64_d7(A, splits, lds, st);
    case 8: return launch_obj64_d8(A, splits, lds, st);
    default: return launch_obj64_d0(A, splits, lds, st);
  }
}

// Reduces the per-split partial keys. mode 0: lower bound (rounded down),
// mode 1: float32 objective (rounded up).
// One wavefront per node (blocks [0, n_nodes)) and, with candidates, one per
// box (blocks [n_nodes, n_nodes + n_boxes)): lanes stride over the splits'
// partial keys, a shuffle reduction combines them. Max / min of packed keys
// does not depend on the order, so the result is the serial reduction's.
__global__ __launch_bounds__(64) void k_bound_finalize(
    const uint64_t *part_key, int n_nodes, int splits, const uint64_t *part_cand, int n_boxes,
    int mode, double rel, double abs_, float *val_raw, double *val_bound, int64_t *argmax,
    int64_t *cand) {
  const int b = blockIdx.x, lane = threadIdx.x;
  if (b < n_nodes) {
    uint64_t key = 0;
    for (int sp = lane; sp < splits; sp += 64) {
      const uint64_t v = part_key[(int64_t)sp * n_nodes + b];
      key = v > key ? v : key;
    }
    key = kcd::wave_max_u64(key);
    if (lane != 0) return;
    const float v = key ? __uint_as_float((uint32_t)(key >> 32)) : 0.0f;
    const uint32_t idx = key ? ~(uint32_t)(key & 0xffffffffu) : 0u;
    if (val_raw) val_raw[b] = v;
    // index 0xffffffff: a screened set settled by its floor alone (no sample)
    if (argmax) argmax[b] = idx == 0xffffffffu ? -1 : (int64_t)idx;
    if (val_bound) {
      const double vd = (double)v;
      double r;
      if (mode == 0) {
        r = vd * (1.0 - rel) - abs_;
        r = r > 0.0 ? r : 0.0;
      } else {
        r = vd * (1.0 + rel) + abs_;
      }
      val_bound[b] = r;
    }
  } else {
    const int i = b - n_nodes;
    if (!cand || i >= n_boxes) return;
    uint64_t key = ~0ull;
    for (int sp = lane; sp < splits; sp += 64) {
      const uint64_t v = part_cand[(int64_t)sp * n_boxes + i];
      key = v < key ? v : key;
    }
    key = kcd::wave_min_u64(key);
    if (lane == 0) cand[i] = key == ~0ull ? -1 : (int64_t)(uint32_t)(key & 0xffffffffu);
  }
}

// One wavefront per candidate set: larger value wins, then the lower index.
__global__ __launch_bounds__(64) void k_obj64_finalize(const double *part_val,
                                                       const uint32_t *part_idx, int n_sets,
                                                       int splits, double *obj, int64_t *argmax) {
  const int c = blockIdx.x, lane = threadIdx.x;
  if (c >= n_sets) return;
  double best = -1.0;
  uint32_t bi = 0xffffffffu;
  for (int sp = lane; sp < splits; sp += 64) {
    const double v = part_val[(int64_t)sp * n_sets + c];
    const uint32_t ii = part_idx[(int64_t)sp * n_sets + c];
    if (v > best || (v == best && ii < bi)) {
      best = v;
      bi = ii;
    }
  }
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    const double ov = __shfl_xor(best, m);
    const uint32_t oi = __shfl_xor(bi, m);
    if (ov > best || (ov == best && oi < bi)) {
      best = ov;
      bi = oi;
    }
  }
  if (lane != 0) return;
  if (obj) obj[c] = best;
  if (argmax) argmax[c] = bi == 0xffffffffu ? -1 : (int64_t)bi;
}

}  // namespace kcb

using namespace kcb;

static int dmax_of(int d) { return d <= 8 ? d : 16; }

// Tile decisions classify one (node, box) pair per lane: 2^lg_kp(k_max) lanes
// per node, so a variant with NG nodes per workgroup needs NG << lg <= 64.
static int lg_kp(int k_max) {
  int lg = 0;
  while ((1 << lg) < k_max && lg < 6) ++lg;
  return lg;
}
static bool ts_fits(int NG, int k_max) { return (NG << lg_kp(k_max)) <= 64; }

static int cand_kc(int k_max) {
  if (k_max <= 4) return 4;
  if (k_max <= 8) return 8;
  if (k_max <= 16) return 16;
  return 64;
}

std::vector<kc_tile> kc_bound_variants(int d, bool with_cand, int k_max) {
  std::vector<kc_tile> v;
  const bool ts = d >= 1 && d <= 8;  // tile decisions are compiled for 1..8 attributes
  if (with_cand) {
    const int kc = cand_kc(k_max);
#define KCB_T3(SV, NGV, KCV) \
  if (KCV == kc) v.push_back({SV, NGV, 8, 0});
    KCB_CAND_VARIANTS(KCB_T3)
#undef KCB_T3
#define KCB_T3S(SV, NGV, KCV) \
  if (KCV == kc && ts && ts_fits(NGV, k_max)) v.push_back({SV, NGV, 8, 1});
    KCB_CAND_TS_VARIANTS(KCB_T3S)
#undef KCB_T3S
  } else {
#define KCB_T2(SV, NGV) v.push_back({SV, NGV, 8, 0});
    KCB_LB_VARIANTS(KCB_T2)
#undef KCB_T2
#define KCB_T2S(SV, NGV) \
  if (ts && ts_fits(NGV, k_max)) v.push_back({SV, NGV, 8, 1});
    KCB_LB_TS_VARIANTS(KCB_T2S)
#undef KCB_T2S
  }
  // each shape at two occupancies; the tile-decision kernels also with
  // smaller splits (more workgroups), since their work per split is uneven
  const size_t n0 = v.size();
  for (size_t i = 0; i < n0; ++i) v.push_back({v[i].S, v[i].NG, 4, v[i].skip});
  for (size_t i = 0; i < n0; ++i)
    if (v[i].skip) {
      v.push_back({v[i].S, v[i].NG, 16, 1});
      v.push_back({v[i].S, v[i].NG, 32, 1});
    }
  return v;
}

static bool cand_compiled(int S, int NG, int KC, int skip, int d) {
  if (skip) {
    if (d < 1 || d > 8) return false;
#define KCB_T4S(SV, NGV, KCV) \
  if (S == SV && NG == NGV && KC == KCV) return true;
    KCB_CAND_TS_VARIANTS(KCB_T4S)
#undef KCB_T4S
    return false;
  }
#define KCB_T4(SV, NGV, KCV) \
  if (S == SV && NG == NGV && KC == KCV) return true;
  KCB_CAND_VARIANTS(KCB_T4)
#undef KCB_T4
  return false;
}

static bool pt_compiled(int S, int NG, int skip) {
  if (skip) {
#define KCB_T7S(SV, NGV) \
  if (S == SV && NG == NGV) return true;
    KCB_PT_TS_VARIANTS(KCB_T7S)
#undef KCB_T7S
    return false;
  }
#define KCB_T7(SV, NGV) \
  if (S == SV && NG == NGV) return true;
  KCB_PT_VARIANTS(KCB_T7)
#undef KCB_T7
  return false;
}

static bool lb_compiled(int S, int NG, int skip, int d) {
  if (skip) {
    if (d < 1 || d > 8) return false;
#define KCB_T5S(SV, NGV) \
  if (S == SV && NG == NGV) return true;
    KCB_LB_TS_VARIANTS(KCB_T5S)
#undef KCB_T5S
    return false;
  }
#define KCB_T5(SV, NGV) \
  if (S == SV && NG == NGV) return true;
  KCB_LB_VARIANTS(KCB_T5)
#undef KCB_T5
  return false;
}

// Candidate variants keep NG x KC running minima per lane; the default holds
// 32 of them (NG = 32 / KC nodes per workgroup, fewer for small batches).
static kc_tile cand_default(int n_nodes, int k_max) {
  const int kc = cand_kc(k_max);
  // 5..8 boxes: four samples per lane and two nodes per workgroup (the
  // autotuner's choice on batched children at D = 4, K = 5)
  if (kc == 8 && n_nodes >= 2) return {4, 2, 8};
  int ng = kc >= 64 ? 1 : 32 / kc;
  while (ng > 1 && ng / 2 >= n_nodes) ng /= 2;
  while (ng > 1 && !cand_compiled(kc >= 16 ? 1 : 2, ng, kc, 0, 0)) ng /= 2;
  return {kc >= 16 ? 1 : 2, ng, 8};
}

kc_tile kc_default_tile(kc_handle *h, int d, bool with_cand, int n_nodes, int k_max, int64_t n) {
  (void)h;
  (void)n;
  if (with_cand) return cand_default(n_nodes, k_max);
  if (n_nodes == 1) return {d <= 4 ? 8 : 4, 1, 8};
  if (n_nodes <= 3) return {4, 2, 8};
  if (n_nodes <= 7) return {4, 4, 8};
  return {d <= 4 ? 4 : 2, 8, 8};
}

__global__ void k_zero_u32(uint32_t *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Shared tile-decision values start below every W and above every cw.
__global__ void k_share_init(uint32_t *gW, int n_nodes, uint32_t *gC, int n_boxes) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_nodes) gW[i] = kcd::FORD_NEG_INF;
  if (gC && i < n_boxes) gC[i] = kcd::FORD_POS_INF;
}

kc_status kc_launch_bound(kc_handle *h, const kc_points *p, int mode, int n_nodes, int n_boxes,
                          int k_max, const int32_t *box_off, const float *lo, const float *hi,
                          float *val_raw, double *val_bound, int64_t *argmax, int64_t *cand,
                          const kc_tile &t0, hipStream_t st, void *fixed_scratch,
                          size_t fixed_bytes, float cut, const double *floor,
                          const float *wit_x, const int64_t *wit_id) {
  const bool point = mode == 1;
  const bool with_cand = cand != nullptr && !point;
  kc_tile t = t0;
  const int DM = dmax_of(p->d);
  const int KC = with_cand ? cand_kc(k_max) : 0;
  if (t.skip && !ts_fits(t.NG, k_max)) t.skip = 0;
  if (with_cand && !cand_compiled(t.S, t.NG, KC, t.skip, p->d)) t = cand_default(n_nodes, k_max);
  if (!with_cand && !point && !lb_compiled(t.S, t.NG, t.skip, p->d))
    t = kc_default_tile(h, p->d, false, n_nodes, k_max, p->n);
  if (point) {
    // the float32 objective: (S, NG) of KCB_PT_VARIANTS, or of
    // KCB_PT_TS_VARIANTS with tile decisions for 1..8 attributes
    if (p->d < 1 || p->d > 8 || !ts_fits(t.NG, k_max)) t.skip = 0;
    if (!pt_compiled(t.S, t.NG, t.skip))
      t = n_nodes <= 2 ? kc_tile{4, 1, t.bpc, 0} : kc_tile{2, 4, t.bpc, 0};
  }
  size_t lds = (size_t)t.NG * k_max * 2 * DM * sizeof(float);
  while (lds > h->lds_per_block && t.NG > 1) {
    t.NG /= 2;
    lds = (size_t)t.NG * k_max * 2 * DM * sizeof(float);
  }
  KC_RETURN_IF(lds > h->lds_per_block, h, KC_EUNSUPPORTED, "boxes of one node exceed LDS");
  const int n_groups = (n_nodes + t.NG - 1) / t.NG;
  const int64_t tile = (int64_t)WG * t.S;
  const int64_t target = (int64_t)h->n_cu * (t.bpc > 0 ? t.bpc : 8);
  int64_t splits = (target + n_groups - 1) / n_groups;
  if (splits < 1) splits = 1;
  int64_t span = (p->n + splits - 1) / splits;
  span = (span + tile - 1) / tile * tile;
  splits = (p->n + span - 1) / span;
  const int64_t grid = splits * n_groups;
  KC_RETURN_IF(grid > 0x7fffffff, h, KC_EUNSUPPORTED, "grid too large");

  const bool screen = point && cut < INFINITY;
  const size_t part_bytes = (size_t)splits * n_nodes * 8;
  const size_t cand_bytes = with_cand ? (size_t)splits * n_boxes * 8 : 0;
  const size_t dead_bytes = screen ? (((size_t)n_nodes * 4 + 255) & ~(size_t)255) : 0;
  const size_t gw_bytes = t.skip ? (((size_t)n_nodes * 4 + 255) & ~(size_t)255) : 0;
  const size_t gc_bytes = t.skip && with_cand ? (((size_t)n_boxes * 4 + 255) & ~(size_t)255) : 0;
  const size_t share_bytes = dead_bytes + gw_bytes + gc_bytes;
  void *scr = nullptr;
  kc_status s = KC_OK;
  if (fixed_scratch) {
    KC_RETURN_IF(screen, h, KC_EINVAL, "screening needs the handle's scratch");
    KC_RETURN_IF(share_bytes + part_bytes + cand_bytes > fixed_bytes, h, KC_EINVAL,
                 "request needs %zu bytes of scratch, above the %zu-byte static scratch of the "
                 "no-allocation entry point (use fewer nodes or boxes per call)",
                 share_bytes + part_bytes + cand_bytes, fixed_bytes);
    scr = fixed_scratch;
  } else if ((s = kc_get_scratch(h, share_bytes + part_bytes + cand_bytes, &scr)) != KC_OK) {
    return s;
  }

  BoundArgs A;
  A.x = p->x;
  A.n = p->n;
  A.ld = p->ld;
  A.d = p->d;
  A.n_nodes = n_nodes;
  A.n_boxes = n_boxes;
  A.k_max = k_max;
  A.box_off = box_off;
  A.lo = lo;
  A.hi = hi;
  A.n_groups = n_groups;
  A.span = span;
  A.lg_kp = lg_kp(k_max);
  A.cut = cut;
  A.dead = nullptr;
  A.floor = point ? floor : nullptr;
  A.wit_x = point && cut < INFINITY ? wit_x : nullptr;
  A.wit_id = point && cut < INFINITY ? wit_id : nullptr;
  A.frel = 2.0 * kc_rel_margin(p->d);
  A.fabs_ = 2.0 * kc_abs_margin(p->d);
  A.gW = A.gC = nullptr;
  if (screen) {
    A.dead = (uint32_t *)scr;
    scr = (char *)scr + dead_bytes;
    k_zero_u32<<<(n_nodes + 255) / 256, 256, 0, st>>>(A.dead, n_nodes);
    if ((s = kc_check_launch(h, "k_zero_u32")) != KC_OK) return s;
  }
  if (t.skip) {
    A.gW = (uint32_t *)scr;
    A.gC = gc_bytes ? (uint32_t *)((char *)scr + gw_bytes) : nullptr;
    scr = (char *)scr + gw_bytes + gc_bytes;
    const int nmax = std::max(n_nodes, gc_bytes ? n_boxes : 0);
    k_share_init<<<(nmax + 255) / 256, 256, 0, st>>>(A.gW, n_nodes, A.gC, gc_bytes ? n_boxes : 0);
    if ((s = kc_check_launch(h, "k_share_init")) != KC_OK) return s;
  }
  A.part_key = (uint64_t *)scr;
  A.part_cand = with_cand ? (uint64_t *)((char *)scr + part_bytes) : nullptr;
  s = dispatch(p->d, t.S, t.NG, KC, point, t.skip, A, (int)grid, lds, st);
  KC_RETURN_IF(s != KC_OK, h, s, "no bound-kernel variant S=%d NG=%d KC=%d point=%d skip=%d", t.S,
               t.NG, KC, (int)point, t.skip);
  s = kc_check_launch(h, "k_bound");
  if (s != KC_OK) return s;
  const int fin = n_nodes + (with_cand ? n_boxes : 0);
  const double rel = kc_rel_margin(p->d) + 0x1p-50;
  k_bound_finalize<<<fin, 64, 0, st>>>(A.part_key, n_nodes, (int)splits,
                                                       A.part_cand, n_boxes, mode, rel,
                                                       kc_abs_margin(p->d), val_raw, val_bound,
                                                       argmax, with_cand ? cand : nullptr);
  return kc_check_launch(h, "k_bound_finalize");
}

// The tile for a lower-bound launch: the autotuner's choice for the shape
// bucket, else the default (the key is built in a stack buffer and looked up
// without allocating).
static kc_tile lb_tile(kc_handle *h, const kc_points *p, const kc_nodes *m, bool cand) {
  char key[96];
  kc_tune_key(key, sizeof(key), p->d, cand, m->n_nodes, m->k_max, p->n);
  auto it = h->tune.find(std::string_view(key));
  if (it != h->tune.end()) return it->second;
  return kc_default_tile(h, p->d, cand, m->n_nodes, m->k_max, p->n);
}

// Tile of the float32 objective (point boxes): the autotuner's choice for the
// shape bucket (attribute count, sets, centers per set, samples), else the
// default.
static void obj_key(char *buf, size_t size, int d, int n_sets, int k, int64_t n) {
  int bn = 0, bs = 0;
  for (int64_t v = n_sets; v > 1; v >>= 1) ++bn;
  for (int64_t v = n; v > 1; v >>= 1) ++bs;
  snprintf(buf, size, "o_d%d_ns%d_k%d_n%d", d, bn, k, bs / 2);
}

kc_tile kc_objective_tile(kc_handle *h, const kc_points *p, int n_sets, int k, bool *tuned) {
  char key[96];
  obj_key(key, sizeof(key), p->d, n_sets, k, p->n);
  auto it = h->tune.find(std::string_view(key));
  if (tuned) *tuned = it != h->tune.end();
  if (it != h->tune.end()) return it->second;
  return n_sets <= 2 ? kc_tile{4, 1, 8} : kc_tile{2, 4, 8};
}

kc_status kc_autotune_objective(kc_handle *h, const kc_points *p, int n_sets, int k,
                                const float *centers, hipStream_t st) {
  double *obj = nullptr;
  int64_t *am = nullptr;
  if (hipMalloc(&obj, (size_t)n_sets * 8) != hipSuccess ||
      hipMalloc(&am, (size_t)n_sets * 8) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(obj);
    return kc_fail(h, KC_ENOMEM, "autotune output buffers");
  }
  std::vector<kc_tile> vars;
#define KCB_T6(SV, NGV) vars.push_back({SV, NGV, 8, 0});
  KCB_PT_VARIANTS(KCB_T6)
#undef KCB_T6
  if (p->d >= 1 && p->d <= 8) {
#define KCB_T6S(SV, NGV)                \
  if (ts_fits(NGV, k)) {                \
    vars.push_back({SV, NGV, 8, 1});    \
    vars.push_back({SV, NGV, 16, 1});   \
    vars.push_back({SV, NGV, 32, 1});   \
  }
    KCB_PT_TS_VARIANTS(KCB_T6S)
#undef KCB_T6S
  }
  double best = 1e30;
  kc_tile bt = kc_objective_tile(h, p, n_sets, k, nullptr);
  kc_status s = KC_OK;
  char key[96];
  obj_key(key, sizeof(key), p->d, n_sets, k, p->n);
  for (const kc_tile &t : vars) {
    double tbest = 1e30;
    for (int rep = 0; rep < 3 && s == KC_OK; ++rep) {
      (void)hipEventRecord(h->ev0, st);
      s = kc_launch_bound(h, p, 1, n_sets, n_sets * k, k, nullptr, centers, centers, nullptr, obj,
                          am, nullptr, t, st);
      (void)hipEventRecord(h->ev1, st);
      if (s != KC_OK) break;
      (void)hipEventSynchronize(h->ev1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, h->ev0, h->ev1);
      if (rep > 0 && ms < tbest) tbest = ms;  // first run is a warm-up
    }
    if (s != KC_OK) break;
    kc_tune_log(key, t, tbest);
    if (tbest < best) {
      best = tbest;
      bt = t;
    }
  }
  (void)hipStreamSynchronize(st);
  (void)hipFree(obj);
  (void)hipFree(am);
  if (s != KC_OK) return s;
  h->tune[key] = bt;
  kc_tune_save(h);
  return KC_OK;
}

bool kc_bound_tuned(kc_handle *h, const kc_points *p, const kc_nodes *m, bool cand) {
  char key[96];
  kc_tune_key(key, sizeof(key), p->d, cand, m->n_nodes, m->k_max, p->n);
  return h->tune.find(std::string_view(key)) != h->tune.end();
}

static kc_status lower_bound_impl(kc_handle *h, const kc_points *pts, const kc_nodes *nodes,
                                  float *lb_raw, double *lb_safe, int64_t *argmax, int64_t *cand,
                                  void *stream, void *fixed_scratch, size_t fixed_bytes) {
  if (!h) return KC_EINVAL;
  kc_status s = kc_validate_points(h, pts);
  if (s != KC_OK) return s;
  s = kc_validate_nodes(h, nodes, pts);
  if (s != KC_OK) return s;
  KC_RETURN_IF(!lb_raw && !lb_safe && !argmax && !cand, h, KC_EINVAL, "no output requested");
  const bool wc = cand != nullptr;
  const kc_tile t = lb_tile(h, pts, nodes, wc);
  return kc_launch_bound(h, pts, 0, nodes->n_nodes, nodes->n_boxes, nodes->k_max, nodes->box_off,
                         nodes->lo, nodes->hi, lb_raw, lb_safe, argmax, cand, t,
                         (hipStream_t)stream, fixed_scratch, fixed_bytes);
}

extern "C" kc_status kc_lower_bound(kc_handle *h, const kc_points *pts, const kc_nodes *nodes,
                                    float *lb_raw, double *lb_safe, int64_t *argmax,
                                    int64_t *cand, void *stream) {
  return kc_guard(h, [&]() -> kc_status {
    return lower_bound_impl(h, pts, nodes, lb_raw, lb_safe, argmax, cand, stream, nullptr, 0);
  });
}

// ------------------------------------------- no-allocation lower bound ------
// Scratch of kc_lower_bound_noalloc: the per-split partial keys of its
// launches. Every GPU the library runs on holds its own copy until the
// process ends. Host code never passes this name to a kernel (on the host it
// is only a stand-in for the symbol): kernels get the device address that
// hipGetSymbolAddress returns, kept per device below. No entry must start at
// zero: every partial key the finalize kernel reads is written by the same
// call's bound kernel first (for well-formed CSR offsets), so the previous
// call's contents never matter. Calls that overlap on one GPU (different
// streams, or several host threads) race on this array.
static __device__ __align__(256) uint64_t scratch[KC_NOALLOC_SCRATCH_BYTES / 8];

static constexpr int kMaxDevices = 64;
static std::atomic<void *> g_scratch_addr[kMaxDevices];

kc_status kc_noalloc_setup(kc_handle *h) {
  KC_RETURN_IF(h->device < 0 || h->device >= kMaxDevices, h, KC_EUNSUPPORTED,
               "device index %d beyond the no-allocation table", h->device);
  void *p = g_scratch_addr[h->device].load();
  if (!p) {
    // h->device is the current device (kc_create set it)
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return kc_fail(h, KC_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    }
    g_scratch_addr[h->device].store(p);
  }
  h->noalloc_scratch = p;
  return KC_OK;
}

extern "C" kc_status kc_lower_bound_noalloc(kc_handle *h, const kc_points *pts,
                                            const kc_nodes *nodes, float *lb_raw, double *lb_safe,
                                            int64_t *argmax, int64_t *cand, void *stream) {
  return kc_guard(h, [&]() -> kc_status {
    if (!h) return KC_EINVAL;
    KC_RETURN_IF(!h->noalloc_scratch, h, KC_EDEVICE, "no static scratch on this device");
    return lower_bound_impl(h, pts, nodes, lb_raw, lb_safe, argmax, cand, stream,
                            h->noalloc_scratch, KC_NOALLOC_SCRATCH_BYTES);
  });
}

extern "C" kc_status kc_objective_screen(kc_handle *h, const kc_points *pts, int32_t n_sets,
                                         int32_t k, const float *centers, float cut,
                                         const double *floor, double *obj, int64_t *argmax,
                                         void *stream) {
  return kc_guard(h, [&]() -> kc_status {
    if (!h) return KC_EINVAL;
    kc_status s = kc_validate_points(h, pts);
    if (s != KC_OK) return s;
    KC_RETURN_IF(n_sets < 1, h, KC_EINVAL, "n_sets must be >= 1 (got %d)", n_sets);
    KC_RETURN_IF(k < 1 || k > 64, h, KC_EINVAL, "k must be in [1,64] (got %d)", k);
    KC_RETURN_IF(!centers, h, KC_EINVAL, "centers is NULL");
    KC_RETURN_IF(std::isnan(cut), h, KC_EINVAL, "cut is NaN");
    KC_RETURN_IF(!obj && !argmax, h, KC_EINVAL, "no output requested");
    const kc_tile t = kc_objective_tile(h, pts, n_sets, k, nullptr);
    return kc_launch_bound(h, pts, 1, n_sets, n_sets * k, k, nullptr, centers, centers, nullptr,
                           obj, argmax, nullptr, t, (hipStream_t)stream, nullptr, 0, cut, floor);
  });
}

kc_status kc_objective_screen_witness(kc_handle *h, const kc_points *pts, int n_sets, int k,
                                      const float *centers, float cut, const double *floor,
                                      const float *wit_x, const int64_t *wit_id, double *obj,
                                      int64_t *argmax, hipStream_t st) {
  const kc_tile t = kc_objective_tile(h, pts, n_sets, k, nullptr);
  return kc_launch_bound(h, pts, 1, n_sets, n_sets * k, k, nullptr, centers, centers, nullptr, obj,
                         argmax, nullptr, t, st, nullptr, 0, cut, floor, wit_x, wit_id);
}

extern "C" kc_status kc_objective(kc_handle *h, const kc_points *pts, int32_t n_sets, int32_t k,
                                  const float *centers, int32_t precision, double *obj,
                                  int64_t *argmax, void *stream) {
  return kc_guard(h, [&]() -> kc_status {
    if (!h) return KC_EINVAL;
    kc_status s = kc_validate_points(h, pts);
    if (s != KC_OK) return s;
    KC_RETURN_IF(n_sets < 1, h, KC_EINVAL, "n_sets must be >= 1 (got %d)", n_sets);
    KC_RETURN_IF(k < 1 || k > 64, h, KC_EINVAL, "k must be in [1,64] (got %d)", k);
    KC_RETURN_IF(!centers, h, KC_EINVAL, "centers is NULL");
    KC_RETURN_IF(precision != 32 && precision != 64, h, KC_EINVAL, "precision must be 32 or 64");
    KC_RETURN_IF(!obj && !argmax, h, KC_EINVAL, "no output requested");
    hipStream_t st = (hipStream_t)stream;
    if (precision == 32) {
      const kc_tile t = kc_objective_tile(h, pts, n_sets, k, nullptr);
      return kc_launch_bound(h, pts, 1, n_sets, n_sets * k, k, nullptr, centers, centers, nullptr,
                             obj, argmax, nullptr, t, st);
    }
    const int DM = dmax_of(pts->d);
    const int64_t target = (int64_t)h->n_cu * 8;
    int64_t splits = (target + n_sets - 1) / n_sets;
    int64_t span = (pts->n + splits - 1) / splits;
    span = (span + WG - 1) / WG * WG;
    splits = (pts->n + span - 1) / span;
    KC_RETURN_IF(n_sets > 65535, h, KC_EUNSUPPORTED, "too many sets for the float64 objective");
    const size_t vb = (size_t)splits * n_sets * sizeof(double);
    const size_t ib = (size_t)splits * n_sets * sizeof(uint32_t);
    void *scr = nullptr;
    s = kc_get_scratch(h, vb + ib, &scr);
    if (s != KC_OK) return s;
    Obj64Args A;
    A.x = pts->x;
    A.n = pts->n;
    A.ld = pts->ld;
    A.d = pts->d;
    A.n_sets = n_sets;
    A.k = k;
    A.centers = centers;
    A.span = span;
    A.part_val = (double *)scr;
    A.part_idx = (uint32_t *)((char *)scr + vb);
    const size_t lds = (size_t)k * DM * sizeof(double);
    s = dispatch64(pts->d, A, (int)splits, lds, st);
    if (s != KC_OK) return kc_fail(h, s, "float64 objective launch");
    s = kc_check_launch(h, "k_obj64");
    if (s != KC_OK) return s;
    k_obj64_finalize<<<n_sets, 64, 0, st>>>(A.part_val, A.part_idx, n_sets, (int)splits, obj,
                                             argmax);
    return kc_check_launch(h, "k_obj64_finalize");
  });
}
