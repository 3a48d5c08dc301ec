// kc_tighten.hip -- kc_tighten / kc_autotune_tighten entry points: launch
// sizing, the tile (samples per lane, nodes per workgroup, occupancy) from the
// autotuner's table, and the kernels that initialise and decode the
// aggregates. The tightening kernel itself is in kc_tighten_impl.h.
#include <cmath>
#include <cstdio>

#include "kc_tighten_impl.h"

namespace kct {
bool launch_tighten_d0(int, int, int, int, int, bool, const TightenArgs &, int, size_t, hipStream_t);
bool launch_tighten_d1(int, int, int, int, int, bool, const TightenArgs &, int, size_t, hipStream_t);
bool launch_tighten_d2(int, int, int, int, int, bool, const TightenArgs &, int, size_t, hipStream_t);
bool launch_tighten_d3(int, int, int, int, int, bool, const TightenArgs &, int, size_t, hipStream_t);
bool launch_tighten_d4(int, int, int, int, int, bool, const TightenArgs &, int, size_t, hipStream_t);
bool launch_tighten_d5(int, int, int, int, int, bool, const TightenArgs &, int, size_t, hipStream_t);
bool launch_tighten_d6(int, int, int, int, int, bool, const TightenArgs &, int, size_t, hipStream_t);
bool launch_tighten_d7(int, int, int, int, int, bool, const TightenArgs &, int, size_t, hipStream_t);
bool launch_tighten_d8(int, int, int, int, int, bool, const TightenArgs &, int, size_t, hipStream_t);

static bool dispatch(int d, int kc, int S, int NG, int minw, int skip, bool refs,
                     const TightenArgs &A, int grid, size_t lds, hipStream_t st) {
  switch (d) {
    case 1: return launch_tighten_d1(kc, S, NG, minw, skip, refs, A, grid, lds, st);
    case 2: return launch_tighten_d2(kc, S, NG, minw, skip, refs, A, grid, lds, st);
    case 3: return launch_tighten_d3(kc, S, NG, minw, skip, refs, A, grid, lds, st);
    case 4: return launch_tighten_d4(kc, S, NG, minw, skip, refs, A, grid, lds, st);
    case 5: return launch_tighten_d5(kc, S, NG, minw, skip, refs, A, grid, lds, st);
    case 6: return launch_tighten_d6(kc, S, NG, minw, skip, refs, A, grid, lds, st);
    case 7: return launch_tighten_d7(kc, S, NG, minw, skip, refs, A, grid, lds, st);
    case 8: return launch_tighten_d8(kc, S, NG, minw, skip, refs, A, grid, lds, st);
    default: return launch_tighten_d0(kc, S, NG, minw, skip, refs, A, grid, lds, st);
  }
}

__global__ void k_tighten_init(uint32_t *bb_lo, uint32_t *bb_hi, uint32_t *amn, uint32_t *amx,
                               uint32_t *n_in, uint32_t *n_asg, uint64_t *far, int64_t nbd, int nb,
                               uint32_t *n_excl, int nn) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nbd) {
    bb_lo[i] = kcd::FORD_POS_INF;
    amn[i] = kcd::FORD_POS_INF;
    bb_hi[i] = kcd::FORD_NEG_INF;
    amx[i] = kcd::FORD_NEG_INF;
  }
  if (i < nb) {
    n_in[i] = 0;
    n_asg[i] = 0;
    if (far) far[i] = 0;
  }
  if (i < nn) n_excl[i] = 0;
}

__global__ void k_tighten_decode(uint32_t *a, uint32_t *b, uint32_t *c, uint32_t *e, int64_t nbd,
                                 uint64_t *far, int nb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nbd) {
    a[i] = __float_as_uint(kcd::fdec(a[i]));
    b[i] = __float_as_uint(kcd::fdec(b[i]));
    c[i] = __float_as_uint(kcd::fdec(c[i]));
    e[i] = __float_as_uint(kcd::fdec(e[i]));
  }
  if (far && i < nb) {
    const uint64_t k = far[i];
    reinterpret_cast<int64_t *>(far)[i] = k ? (int64_t)(~(uint32_t)(k & 0xffffffffu)) : -1;
  }
}

// ---------------------------------------------------------------------------
// Inside-only tightening. In a batch without refs, a node of two or more
// boxes whose center-based bound stays within alpha for every box over a set
// of samples excludes none of them from any box, so none is assigned or
// excluded (their label is -1, Algorithm 3) and they belong to S_+^k exactly
// when they lie inside box k (Algorithm 4 without refs). For such (node,
// chunk of LCHUNK samples) pairs only the inside test and the bounding-box
// fold are needed: k_tighten_inside does them, with a fraction of the full
// kernel's registers and instructions, and marks the pair in a map that the
// full kernel reads to skip it. k_chunk_bbox gives each chunk's bounding
// box; the decision applies the per-sample operations in the same order to
// the bounding box's extreme coordinates (float32 rounding is monotone, so
// no sample's bound exceeds the chunk's).

__global__ __launch_bounds__(256) void k_chunk_bbox(const float *x, int64_t n, int64_t ld, int d,
                                                    float *cbb) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ uint32_t s_lo[4][16], s_hi[4][16];
  const int64_t c0 = (int64_t)blockIdx.x * LCHUNK;
  for (int a = 0; a < d; ++a) {
    const float *p = x + (int64_t)a * ld;
    float l = INFINITY, h = -INFINITY;
#pragma unroll
    for (int j = 0; j < LCHUNK / 256; ++j) {
      const int64_t i = c0 + j * 256 + tid;
      if (i < n) {
        l = fminf(l, p[i]);
        h = fmaxf(h, p[i]);
      }
    }
    const uint32_t wl = kcd::wave_min_u32(kcd::ford(l)), wh = kcd::wave_max_u32(kcd::ford(h));
    if (lane == 0) {
      s_lo[wave][a] = wl;
      s_hi[wave][a] = wh;
    }
  }
  __syncthreads();
  if (tid < d) {
    uint32_t l = s_lo[0][tid], h = s_hi[0][tid];
    for (int w = 1; w < 4; ++w) {
      l = min(l, s_lo[w][tid]);
      h = max(h, s_hi[w][tid]);
    }
    cbb[((int64_t)blockIdx.x * 2) * d + tid] = kcd::fdec(l);
    cbb[((int64_t)blockIdx.x * 2 + 1) * d + tid] = kcd::fdec(h);
  }
}

// NG nodes and one split of whole chunks per workgroup: per chunk, each
// node's decision from the chunk's bounding box; when it holds for some node,
// the chunk's samples are read once and, per lane, the count and bounding box
// of its samples inside each box of those nodes are folded.
template <int D, int KC, int S, int NG>
__global__ __launch_bounds__(WG) void k_tighten_inside(TightenArgs A, const float *cbb,
                                                       uint8_t *map, int64_t chunks_per_split) {
  __shared__ float sb[NG][KC][2][D];
  __shared__ int s_b0[NG], s_cnt[NG];
  const int tid = threadIdx.x, lane = tid & 63;
  const int u = kcd::xcd_unit(blockIdx.x, gridDim.x);
  const int n_groups = (A.n_nodes + NG - 1) / NG;
  const int grp = u % n_groups, split = u / n_groups;
  const int m0 = grp * NG;
  if (tid < NG) {
    const int m = m0 + tid;
    int b0 = 0, c = 0;
    if (m < A.n_nodes) {
      b0 = kcd::clampi(A.box_off[m], 0, A.n_boxes);
      const int b1 = kcd::clampi(A.box_off[m + 1], b0, A.n_boxes);
      c = min(min(b1 - b0, A.k_max), KC);
    }
    s_b0[tid] = b0;
    s_cnt[tid] = c;
  }
  __syncthreads();
  for (int i = tid; i < NG * KC * D; i += WG) {
    const int jn = i / (KC * D), r = i - jn * KC * D;
    const int k = r / D, a = r - k * D;
    const bool ok = k < s_cnt[jn];
    sb[jn][k][0][a] = ok ? A.lo[(int64_t)(s_b0[jn] + k) * D + a] : 0.f;
    sb[jn][k][1][a] = ok ? A.hi[(int64_t)(s_b0[jn] + k) * D + a] : 0.f;
  }
  __syncthreads();
  float bmin[NG][KC][D], bmax[NG][KC][D];
  uint32_t nin[NG][KC];
#pragma unroll
  for (int jn = 0; jn < NG; ++jn)
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      nin[jn][k] = 0;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        bmin[jn][k][a] = INFINITY;
        bmax[jn][k][a] = -INFINITY;
      }
    }
  const int64_t cb0 = (int64_t)split * chunks_per_split;
  const int64_t cb1 = min(A.n_lchunks, cb0 + chunks_per_split);
  for (int64_t c = cb0; c < cb1; ++c) {
    // each node's decision for the chunk (uniform): every box's center-based
    // bound over the chunk's bounding box within alpha
    uint32_t lightm = 0;
#pragma unroll
    for (int jn = 0; jn < NG; ++jn) {
      const int cnt = s_cnt[jn];
      bool light = m0 + jn < A.n_nodes && cnt >= 2;
      for (int k = 0; k < cnt && light; ++k) {
        float ub = 0.f;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          const float blo = cbb[(c * 2) * D + a], bhi = cbb[(c * 2 + 1) * D + a];
          const float uu = fmaxf(fmaxf(sb[jn][k][0][a] - blo, bhi - sb[jn][k][1][a]), 0.f);
          ub = (a == 0) ? uu * uu : __builtin_fmaf(uu, uu, ub);
        }
        light = !(ub > A.t_center);
      }
      if (tid == 0 && m0 + jn < A.n_nodes) map[(int64_t)(m0 + jn) * A.n_lchunks + c] = light ? 1 : 0;
      if (light) lightm |= 1u << jn;
    }
    if (!lightm) continue;
    const int64_t s_hi = min(A.n, (c + 1) * (int64_t)LCHUNK);
    for (int64_t base = c * (int64_t)LCHUNK + (int64_t)tid * S; base < s_hi;
         base += (int64_t)WG * S) {
      float xs[S][D];
      const bool full = base + S <= s_hi;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const float *p = A.x + (int64_t)a * A.ld + base;
        if (full && S == 4) {
          const float4 v = *reinterpret_cast<const float4 *>(p);
          xs[0][a] = v.x;
          xs[1 % S][a] = v.y;
          xs[2 % S][a] = v.z;
          xs[3 % S][a] = v.w;
        } else if (full && S == 2) {
          const float2 v = *reinterpret_cast<const float2 *>(p);
          xs[0][a] = v.x;
          xs[1 % S][a] = v.y;
        } else {
#pragma unroll
          for (int i = 0; i < S; ++i) xs[i][a] = (base + i < s_hi) ? p[i] : 0.f;
        }
      }
#pragma unroll
      for (int jn = 0; jn < NG; ++jn) {
        if (!((lightm >> jn) & 1u)) continue;
        const int cnt = s_cnt[jn];
#pragma unroll
        for (int k = 0; k < KC; ++k) {
          if (k >= cnt) break;
          float l[D], h[D];
#pragma unroll
          for (int a = 0; a < D; ++a) {
            l[a] = sb[jn][k][0][a];
            h[a] = sb[jn][k][1][a];
          }
#pragma unroll
          for (int i = 0; i < S; ++i) {
            bool in = base + i < s_hi;
#pragma unroll
            for (int a = 0; a < D; ++a) in = in && l[a] <= xs[i][a] && xs[i][a] <= h[a];
            if (in) {
              ++nin[jn][k];
#pragma unroll
              for (int a = 0; a < D; ++a) {
                bmin[jn][k][a] = fminf(bmin[jn][k][a], xs[i][a]);
                bmax[jn][k][a] = fmaxf(bmax[jn][k][a], xs[i][a]);
              }
            }
          }
        }
      }
    }
  }
#pragma unroll
  for (int jn = 0; jn < NG; ++jn) {
    const int cnt = m0 + jn < A.n_nodes ? s_cnt[jn] : 0;
    const int b0 = s_b0[jn];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const uint32_t ci = kcd::wave_sum_u32(nin[jn][k]);
      if (!ci) continue;  // uniform
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const uint32_t v0 = kcd::wave_min_u32(kcd::ford(bmin[jn][k][a]));
        const uint32_t v1 = kcd::wave_max_u32(kcd::ford(bmax[jn][k][a]));
        if (lane == 0 && k < cnt) {
          const int64_t o = (int64_t)(b0 + k) * D + a;
          atomicMin(&A.bb_lo[o], v0);
          atomicMax(&A.bb_hi[o], v1);
        }
      }
      if (lane == 0 && k < cnt) atomicAdd(&A.n_in[b0 + k], ci);
    }
  }
}

// Nodes per workgroup of the inside-only kernel: as many as keep its
// per-lane aggregates within about 96 registers.
static int inside_ng(int d, int kc) {
  const int per = 2 * kc * d + kc;
  return per * 4 <= 96 ? 4 : (per * 2 <= 96 ? 2 : 1);
}

template <int D>
static bool launch_inside_d(int kc, const TightenArgs &A, const float *cbb, uint8_t *map,
                            int64_t cps, int grid, hipStream_t st) {
  constexpr int S = D <= 4 ? 4 : 2;
  const int ng = inside_ng(D, kc);
#define KCT_IN(KV)                                                                      \
  case KV:                                                                              \
    if (ng == 4)                                                                        \
      k_tighten_inside<D, KV, S, 4><<<grid, WG, 0, st>>>(A, cbb, map, cps);              \
    else if (ng == 2)                                                                   \
      k_tighten_inside<D, KV, S, 2><<<grid, WG, 0, st>>>(A, cbb, map, cps);              \
    else                                                                                \
      k_tighten_inside<D, KV, S, 1><<<grid, WG, 0, st>>>(A, cbb, map, cps);              \
    return true;
  switch (kc) {
    KCT_IN(1) KCT_IN(2) KCT_IN(3) KCT_IN(4) KCT_IN(5) KCT_IN(6) KCT_IN(8)
    default: return false;
  }
#undef KCT_IN
}

static bool launch_inside(int d, int kc, const TightenArgs &A, const float *cbb, uint8_t *map,
                          int64_t cps, int grid, hipStream_t st) {
  switch (d) {
    case 1: return launch_inside_d<1>(kc, A, cbb, map, cps, grid, st);
    case 2: return launch_inside_d<2>(kc, A, cbb, map, cps, grid, st);
    case 3: return launch_inside_d<3>(kc, A, cbb, map, cps, grid, st);
    case 4: return launch_inside_d<4>(kc, A, cbb, map, cps, grid, st);
    case 5: return launch_inside_d<5>(kc, A, cbb, map, cps, grid, st);
    case 6: return launch_inside_d<6>(kc, A, cbb, map, cps, grid, st);
    case 7: return launch_inside_d<7>(kc, A, cbb, map, cps, grid, st);
    case 8: return launch_inside_d<8>(kc, A, cbb, map, cps, grid, st);
    default: return false;
  }
}

static const int kKC[] = {1, 2, 3, 4, 5, 6, 8};

// Boxes per chunk: all boxes of a node when their aggregates fit in about 160
// registers, else the largest compiled chunk that does.
static int choose_kc(int d, int k_max) {
  const int DM = d <= 8 ? d : 16;
  const int cap = d > 8 ? 2 : 8;
  int best = 1;
  for (int c : kKC) {
    if (c > cap || c * (4 * DM + 4) > 160) break;
    best = c;
    if (c >= k_max) break;
  }
  return best;
}

static int dsupp(int d) { return d <= 8 ? d : 0; }

static int lg_kp(int k_max) {
  int lg = 0;
  while ((1 << lg) < k_max && lg < 6) ++lg;
  return lg;
}

// The compiled tiles (S, NG, occupancy, tile decisions) for this attribute
// count and chunk (the same table as launch_kc in kc_tighten_impl.h); skip 2
// is the wide kernel (kc_tighten_wide.h), for NG << lg_kp(k_max) <= 64.
static std::vector<kc_tile> tighten_variants(int d, int kc, bool single, int k_max) {
  const int D = dsupp(d);
  const int SD = D > 0 && D <= 4 ? 4 : 2;
  const int MD = D > 0 && D * kc <= 6 ? 6 : 0;
  const int MA = MD == 4 ? 2 : 4;
  std::vector<kc_tile> v{{SD, 1, MD, 0}, {SD, 1, MA, 0}, {SD / 2, 1, MD, 0}};
  if (single && D > 0 && D * kc <= 20) v.push_back({SD, 2, 0, 0});
  if (single && D > 0) {
    for (int m : {1, 2, 4}) v.push_back({m * SD, 1, 0, 1});
    if (D * kc <= 20)
      for (int m : {1, 2}) v.push_back({m * SD, 2, 0, 1});
    const int lg = lg_kp(k_max);
// wide tiles: grids of 8 (bpc 0), 3, 16, 32 or 64 workgroups per compute unit
// (smaller splits balance uneven work, fewer are resident at once); bpc
// 1000 + g: a grid of g per compute unit with registers capped at four
// wavefronts per SIMD (S <= 8)
#define KCT_WV(SV, NGV)                                                 \
  if ((NGV << lg) <= 64) {                                              \
    for (int g : {0, 3, 16, 32, 64}) v.push_back({SV, NGV, g, 2});     \
    if (SV <= 8)                                                        \
      for (int g : {4, 32, 64}) v.push_back({SV, NGV, 1000 + g, 2});  \
  }
    KCT_WIDE_VARIANTS(KCT_WV)
#undef KCT_WV
  }
  return v;
}

static bool tile_ok(int d, int kc, bool single, int k_max, const kc_tile &t) {
  for (const kc_tile &v : tighten_variants(d, kc, single, k_max))
    if (v.S == t.S && v.NG == t.NG && v.bpc == t.bpc && v.skip == t.skip) return true;
  return false;
}

// Autotune table key of a tightening launch: attribute count, boxes per node,
// node count and sample count buckets, with or without refs (the tile field
// bpc holds the occupancy of the tightening variant).
static void tighten_key(char *buf, size_t size, int d, int k_max, int n_nodes, int64_t n,
                        bool refs) {
  int bn = 0, bs = 0;
  for (int64_t v = n_nodes; v > 1; v >>= 1) ++bn;
  for (int64_t v = n; v > 1; v >>= 1) ++bs;
  snprintf(buf, size, "t_d%d_k%d_nn%d_n%d_r%d", d, k_max, bn, bs / 2, (int)refs);
}

struct Launch {
  TightenArgs A;
  kc_tile t;  // the tile used (the requested one, unless it does not apply)
  int kc, grid;
  size_t lds;
  bool refs;
  int64_t nbd, nmax;
  bool inside;  // try the inside-only kernel on the (node, chunk) pairs it settles
  int grid_inside;
  int64_t cps, n_lchunks;  // chunks per split of the inside-only kernel; chunks
};

// Validates the request and sizes a launch with tile t (NG > 1 only when all
// boxes of a node fit one chunk and no labels are requested).
static kc_status plan(kc_handle *h, const kc_points *pts, const kc_nodes *nodes, double alpha,
                      const kc_refs *refs, bool labels, kc_tile t, Launch &L) {
  const int d = pts->d, DM = d <= 8 ? d : 16;
  const int kc = choose_kc(d, nodes->k_max);
  const int n_chunks = (nodes->k_max + kc - 1) / kc;
  const bool single = n_chunks == 1 && !labels;
  if (!tile_ok(d, kc, single, nodes->k_max, t)) t = tighten_variants(d, kc, single, nodes->k_max)[0];
  const int max_refs = refs ? refs->max_per_box : 0;
  const int node_floats = nodes->k_max * 4 * DM + nodes->k_max * max_refs * DM;
  // dynamic LDS (node slots) plus the kernel's static node table
  size_t lds = (size_t)t.NG * node_floats * 4;
  if (lds + t.NG * sizeof(NodeSlot) > h->lds_per_block && t.NG > 1) {
    t = tighten_variants(d, kc, single, nodes->k_max)[0];
    lds = (size_t)node_floats * 4;
  }
  KC_RETURN_IF(lds + t.NG * sizeof(NodeSlot) > h->lds_per_block, h, KC_EUNSUPPORTED,
               "boxes and refs of a node exceed LDS");
  const int S = t.S;
  const int n_groups = (nodes->n_nodes + t.NG - 1) / t.NG;
  const int64_t units = (int64_t)n_groups * n_chunks;
  const int64_t target = (int64_t)h->n_cu * (t.skip == 2 && t.bpc % 1000 > 0 ? t.bpc % 1000 : 8);
  int64_t splits = (target + units - 1) / units;
  int64_t span = (pts->n + splits - 1) / splits;
  span = (span + WG * S - 1) / (WG * S) * (WG * S);
  splits = (pts->n + span - 1) / span;
  const int64_t grid = splits * units;
  KC_RETURN_IF(grid > 0x7fffffff, h, KC_EUNSUPPORTED, "grid too large");

  TightenArgs &A = L.A;
  A = TightenArgs{};
  A.x = pts->x;
  A.n = pts->n;
  A.ld = pts->ld;
  A.d = d;
  A.n_nodes = nodes->n_nodes;
  A.n_boxes = nodes->n_boxes;
  A.k_max = nodes->k_max;
  A.box_off = nodes->box_off;
  A.lo = nodes->lo;
  A.hi = nodes->hi;
  A.ref_off = refs ? refs->ref_off : nullptr;
  A.ref = refs ? refs->ref : nullptr;
  A.n_refs = refs ? refs->n_refs : 0;
  A.max_refs = max_refs;
  A.t_center = kc_thr_gt(alpha, d);
  A.t_sample = kc_thr_gt(4.0 * alpha, d);
  A.t_ball = kc_thr_gt(alpha, d);
  A.n_chunks = n_chunks;
  A.kc = kc;
  A.n_groups = n_groups;
  A.node_floats = node_floats;
  A.span = span;
  A.lg_kp = lg_kp(nodes->k_max);
  L.kc = kc;
  L.grid = (int)grid;
  L.lds = lds;
  L.refs = A.ref_off != nullptr;
  L.nbd = (int64_t)nodes->n_boxes * d;
  const int64_t ni = L.nbd > nodes->n_boxes ? L.nbd : nodes->n_boxes;
  L.nmax = ni > nodes->n_nodes ? ni : nodes->n_nodes;
  L.t = t;
  // batched launches without refs whose boxes fit one chunk, 1..8 attributes
  // (the wide kernel settles such tiles itself)
  L.inside = !refs && n_chunks == 1 && !labels && d >= 1 && d <= 8 && nodes->n_nodes >= 8 &&
             t.skip != 2;
  L.grid_inside = 0;
  L.cps = 0;
  if (L.inside) {
    const int64_t nch = (pts->n + LCHUNK - 1) / LCHUNK;
    const int ng = inside_ng(d, kc);
    const int64_t groups = (nodes->n_nodes + ng - 1) / ng;
    int64_t sp = (target + groups - 1) / groups;
    L.cps = (nch + sp - 1) / sp;
    sp = (nch + L.cps - 1) / L.cps;
    L.inside = sp * groups <= 0x7fffffff;
    L.grid_inside = (int)(sp * groups);
    L.n_lchunks = nch;
  }
  return KC_OK;
}

// Initialise, run the tile's kernel, decode; outputs as in kc_tighten.
static kc_status run(kc_handle *h, Launch &L, float *bb_lo, float *bb_hi,
                     uint32_t *n_in, float *asg_min, float *asg_max, uint32_t *n_asg,
                     uint32_t *n_excl, int64_t *asg_far, int8_t *labels, int n_boxes, int n_nodes,
                     hipStream_t st) {
  if (L.nmax > 0)
    k_tighten_init<<<(L.nmax + 255) / 256, 256, 0, st>>>(
        (uint32_t *)bb_lo, (uint32_t *)bb_hi, (uint32_t *)asg_min, (uint32_t *)asg_max, n_in,
        n_asg, (uint64_t *)asg_far, L.nbd, n_boxes, n_excl, n_nodes);
  kc_status s = kc_check_launch(h, "k_tighten_init");
  if (s != KC_OK) return s;
  TightenArgs &A = L.A;
  A.bb_lo = (uint32_t *)bb_lo;
  A.bb_hi = (uint32_t *)bb_hi;
  A.asg_min = (uint32_t *)asg_min;
  A.asg_max = (uint32_t *)asg_max;
  A.n_in = n_in;
  A.n_asg = n_asg;
  A.n_excl = n_excl;
  A.asg_far = (uint64_t *)asg_far;
  A.labels = labels;
  A.light_map = nullptr;
  A.n_lchunks = 0;
  if (L.inside) {
    const int d = A.d;
    const size_t cbb_bytes = ((size_t)L.n_lchunks * 2 * d * 4 + 255) & ~(size_t)255;
    const size_t map_bytes = (size_t)A.n_nodes * L.n_lchunks;
    void *scr = nullptr;
    if ((s = kc_get_scratch(h, cbb_bytes + map_bytes, &scr)) != KC_OK) return s;
    float *cbb = (float *)scr;
    uint8_t *map = (uint8_t *)scr + cbb_bytes;
    k_chunk_bbox<<<(unsigned)L.n_lchunks, 256, 0, st>>>(A.x, A.n, A.ld, d, cbb);
    if ((s = kc_check_launch(h, "k_chunk_bbox")) != KC_OK) return s;
    A.n_lchunks = L.n_lchunks;
    KC_RETURN_IF(!launch_inside(d, L.kc, A, cbb, map, L.cps, L.grid_inside, st), h,
                 KC_EUNSUPPORTED, "no inside-only tighten variant for d=%d kc=%d", d, L.kc);
    if ((s = kc_check_launch(h, "k_tighten_inside")) != KC_OK) return s;
    A.light_map = map;
  }
  const kc_tile &t = L.t;
  KC_RETURN_IF(!dispatch(A.d, L.kc, t.S, t.NG, t.bpc, t.skip, L.refs, A, L.grid, L.lds, st), h,
               KC_EUNSUPPORTED, "no tighten variant for d=%d kc=%d S=%d NG=%d", A.d, L.kc, t.S, t.NG);
  s = kc_check_launch(h, "k_tighten");
  if (s != KC_OK) return s;
  if (L.nmax > 0)
    k_tighten_decode<<<(L.nmax + 255) / 256, 256, 0, st>>>((uint32_t *)bb_lo, (uint32_t *)bb_hi,
                                                           (uint32_t *)asg_min, (uint32_t *)asg_max,
                                                           L.nbd, (uint64_t *)asg_far, n_boxes);
  return kc_check_launch(h, "k_tighten_decode");
}

static kc_status validate(kc_handle *h, const kc_points *pts, const kc_nodes *nodes, double alpha,
                          const kc_refs *refs) {
  kc_status s = kc_validate_points(h, pts);
  if (s != KC_OK) return s;
  s = kc_validate_nodes(h, nodes, pts);
  if (s != KC_OK) return s;
  s = kc_validate_refs(h, refs, nodes);
  if (s != KC_OK) return s;
  KC_RETURN_IF(std::isnan(alpha) || alpha < 0, h, KC_EINVAL, "alpha must be >= 0");
  return KC_OK;
}

}  // namespace kct

using namespace kct;

kc_tile kc_tighten_tile(kc_handle *h, const kc_points *pts, const kc_nodes *nodes,
                        const kc_refs *refs, bool *tuned) {
  char key[96];
  tighten_key(key, sizeof(key), pts->d, nodes->k_max, nodes->n_nodes, pts->n, refs != nullptr);
  auto it = h->tune.find(std::string_view(key));
  if (tuned) *tuned = it != h->tune.end();
  if (it != h->tune.end()) return it->second;
  const int kc = choose_kc(pts->d, nodes->k_max);
  return tighten_variants(pts->d, kc, (nodes->k_max + kc - 1) / kc == 1, nodes->k_max)[0];
}

extern "C" kc_status kc_tighten(kc_handle *h, const kc_points *pts, const kc_nodes *nodes,
                                double alpha, const kc_refs *refs, float *bb_lo, float *bb_hi,
                                uint32_t *n_in, float *asg_min, float *asg_max, uint32_t *n_asg,
                                uint32_t *n_excl, int64_t *asg_far, int8_t *labels, void *stream) {
  return kc_guard(h, [&]() -> kc_status {
    if (!h) return KC_EINVAL;
    kc_status s = validate(h, pts, nodes, alpha, refs);
    if (s != KC_OK) return s;
    KC_RETURN_IF(!bb_lo || !bb_hi || !n_in || !asg_min || !asg_max || !n_asg || !n_excl, h,
                 KC_EINVAL, "an output array is NULL");
    KC_RETURN_IF(labels && nodes->n_nodes != 1, h, KC_EINVAL, "labels need n_nodes == 1");
    Launch L;
    const kc_tile t0 = kc_tighten_tile(h, pts, nodes, refs, nullptr);
    s = plan(h, pts, nodes, alpha, refs, labels != nullptr, t0, L);
    if (s != KC_OK) return s;
    return run(h, L, bb_lo, bb_hi, n_in, asg_min, asg_max, n_asg, n_excl, asg_far, labels,
               nodes->n_boxes, nodes->n_nodes, (hipStream_t)stream);
  });
}

extern "C" kc_status kc_autotune_tighten(kc_handle *h, const kc_points *pts, const kc_nodes *nodes,
                                         double alpha, const kc_refs *refs, double *best_ms,
                                         void *stream) {
  return kc_guard(h, [&]() -> kc_status {
    if (!h) return KC_EINVAL;
    kc_status s = validate(h, pts, nodes, alpha, refs);
    if (s != KC_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const int nb = nodes->n_boxes, nn = nodes->n_nodes, d = pts->d;
    const size_t nbd = (size_t)(nb > 0 ? nb : 1) * d;
    // scratch outputs: four [nb][d] float arrays, two [nb] counts, [nn]
    // exclusions, [nb] farthest keys
    const size_t bytes = nbd * 16 + (size_t)(nb > 0 ? nb : 1) * 16 + (size_t)nn * 4 + 1024;
    char *buf = nullptr;
    if (hipMalloc(&buf, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return kc_fail(h, KC_ENOMEM, "autotune output buffers");
    }
    float *o_bl = (float *)buf, *o_bh = o_bl + nbd, *o_am = o_bh + nbd, *o_ax = o_am + nbd;
    int64_t *o_far = (int64_t *)(((uintptr_t)(o_ax + nbd) + 255) & ~(uintptr_t)255);
    uint32_t *o_ni = (uint32_t *)(o_far + (nb > 0 ? nb : 1));
    uint32_t *o_na = o_ni + (nb > 0 ? nb : 1), *o_ne = o_na + (nb > 0 ? nb : 1);
    const int kc = choose_kc(d, nodes->k_max);
    const bool single = (nodes->k_max + kc - 1) / kc == 1;
    double best = 1e30;
    kc_tile bt = tighten_variants(d, kc, single, nodes->k_max)[0];
    char key[96];
    tighten_key(key, sizeof(key), d, nodes->k_max, nn, pts->n, refs != nullptr);
    for (const kc_tile &t : tighten_variants(d, kc, single, nodes->k_max)) {
      Launch L;
      s = plan(h, pts, nodes, alpha, refs, false, t, L);
      if (s != KC_OK) break;
      if (L.t.S != t.S || L.t.NG != t.NG || L.t.bpc != t.bpc || L.t.skip != t.skip)
        continue;  // did not fit LDS
      double tbest = 1e30;
      for (int rep = 0; rep < 3 && s == KC_OK; ++rep) {
        (void)hipEventRecord(h->ev0, st);
        s = run(h, L, o_bl, o_bh, o_ni, o_am, o_ax, o_na, o_ne, o_far, nullptr, nb, nn, st);
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
    (void)hipFree(buf);
    if (s != KC_OK) return s;
    h->tune[key] = bt;
    kc_tune_save(h);
    if (best_ms) *best_ms = best;
    return KC_OK;
  });
}
