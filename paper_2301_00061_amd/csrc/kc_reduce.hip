// kc_reduce.hip -- sample reduction (Algorithm 5, Section 4.2): per-sample
// redundancy flags over all open nodes, then a stable compaction of the
// structure-of-arrays samples and their original indices.
//
// Three launches: (1) flags + kept count per tile of 1024 samples, (2) one
// workgroup scans the tile counts into tile offsets and the total, (3) every
// tile rebuilds its in-tile ranks from wavefront ballots and scatters the kept
// samples. Order is preserved, so the output is deterministic.
#include <cmath>

#include "kc_device.h"
#include "kc_internal.h"

namespace kcr {

constexpr int WG = 256;
// samples per lane: 16 for 1..4 attributes (fewer workgroups, fewer tile
// decisions per sample), else 4; a workgroup's tile is WG * per_lane(D)
constexpr int per_lane(int D) { return D >= 1 && D <= 4 ? 16 : 4; }
inline int64_t tile_of(int d) { return (int64_t)WG * per_lane(d <= 8 ? d : 0); }

struct FlagArgs {
  const float *x;
  int64_t n, ld;
  int d;
  int n_nodes, n_boxes, k_max;
  const int32_t *box_off;
  const float *lo, *hi;
  const int32_t *ref_off;
  const float *ref;
  int n_refs, max_refs;
  float t_beta;   // alpha_s(M) < t_beta   => LB-redundant in M
  float t_alpha;  // dist > t_alpha        => UB-redundant with that ref
  int lg_kp;      // tile decisions: 2^lg_kp >= k_max lanes per node
  uint8_t *keep;
  uint32_t *tile_cnt;
};

template <int D>
__device__ __forceinline__ bool redundant_in_node(const FlagArgs &A, int m, const float *xv,
                                                  int dd) {
  constexpr int DM = D ? D : 16;
  const int b0 = kcd::clampi(A.box_off[m], 0, A.n_boxes);
  const int b1 = kcd::clampi(A.box_off[m + 1], b0, A.n_boxes);
  const int cnt = min(b1 - b0, A.k_max);
  float as = INFINITY;
  bool ub = true;
  for (int k = 0; k < cnt; ++k) {
    const float *l = A.lo + (int64_t)(b0 + k) * dd;
    const float *h = A.hi + (int64_t)(b0 + k) * dd;
    float acc = 0.f;
    bool in = true;
#pragma unroll
    for (int a = 0; a < DM; ++a) {
      if (a < dd) {
        const float tl = fabsf(xv[a] - l[a]);
        const float th = fabsf(xv[a] - h[a]);
        const float t = fmaxf(tl, th);
        acc = (a == 0) ? t * t : __builtin_fmaf(t, t, acc);
        in = in && (l[a] <= xv[a]) && (xv[a] <= h[a]);
      }
    }
    as = fminf(as, acc);
    if (in) {
      // UB-redundant for this box only if some ref of the box is farther than alpha
      bool far = false;
      if (A.ref_off) {
        const int rb = kcd::clampi(A.ref_off[b0 + k], 0, A.n_refs);
        const int re = kcd::clampi(A.ref_off[b0 + k + 1], rb, A.n_refs);
        const int rc = min(re - rb, A.max_refs);
        for (int r = 0; r < rc; ++r) {
          const float *rr = A.ref + (int64_t)(rb + r) * dd;
          float dq = 0.f;
#pragma unroll
          for (int a = 0; a < DM; ++a) {
            if (a < dd) {
              const float t = xv[a] - rr[a];
              dq = (a == 0) ? t * t : __builtin_fmaf(t, t, dq);
            }
          }
          far = far || (dq > A.t_alpha);
        }
      }
      ub = ub && far;
    }
  }
  return ub && (as < A.t_beta);
}

// Tile decisions: nodes g0 .. g0 + 64/KP - 1 (KP = 2^lg lanes per node, at
// least k_max) classified for a wavefront's tile of samples with bounding box
// [tlo, thi], one (node, box) pair per lane. The bounds over the tile are the
// per-sample operations in the same order on the tile's extreme coordinates;
// float32 rounding is monotone, so a bound on the safe side of a threshold
// gives every sample of the tile the same outcome. Bit (jn << lg) of
// *keep_all: no sample of the tile is redundant in node g0 + jn; of *red_all:
// every sample is (or the node does not exist).
template <int DM>
__device__ __forceinline__ void classify_nodes(const FlagArgs &A, int g0, int lg,
                                               const float (&tlo)[DM], const float (&thi)[DM],
                                               int dd, int lane, uint64_t &keep_all,
                                               uint64_t &red_all) {
  const int KP = 1 << lg;
  const int jn = lane >> lg, k = lane & (KP - 1);
  const int m = g0 + jn;
  const bool node_ok = m < A.n_nodes;
  float alo = INFINITY, ahi = INFINITY;
  bool ub_all = true, ub_none = false;
  if (node_ok) {
    const int b0 = kcd::clampi(A.box_off[m], 0, A.n_boxes);
    const int b1 = kcd::clampi(A.box_off[m + 1], b0, A.n_boxes);
    const int cnt = min(b1 - b0, A.k_max);
    if (k < cnt) {
      const float *l = A.lo + (int64_t)(b0 + k) * dd;
      const float *h = A.hi + (int64_t)(b0 + k) * dd;
      float lacc = 0.f, hacc = 0.f;
      bool in_all = true, in_none = false;
#pragma unroll
      for (int a = 0; a < DM; ++a) {
        if (a < dd) {
          const float la = l[a], ha = h[a];
          // |x - la| and |x - ha| over the tile's range: x - c rounds
          // monotonically in x, so the extremes sit at the range's ends
          const float ul = fmaxf(fabsf(tlo[a] - la), fabsf(thi[a] - la));
          const float uh = fmaxf(fabsf(tlo[a] - ha), fabsf(thi[a] - ha));
          const float gl = fmaxf(fmaxf(tlo[a] - la, la - thi[a]), 0.f);
          const float gh = fmaxf(fmaxf(tlo[a] - ha, ha - thi[a]), 0.f);
          const float tu = fmaxf(ul, uh), tl = fmaxf(gl, gh);
          lacc = (a == 0) ? tl * tl : __builtin_fmaf(tl, tl, lacc);
          hacc = (a == 0) ? tu * tu : __builtin_fmaf(tu, tu, hacc);
          in_all = in_all && la <= tlo[a] && thi[a] <= ha;
          in_none = in_none || thi[a] < la || tlo[a] > ha;
        }
      }
      alo = lacc;
      ahi = hacc;
      if (!in_none) {
        // some ref farther than alpha from the whole tile / every ref within
        // alpha of the whole tile
        bool far_all = false, far_none = true;
        if (A.ref_off) {
          const int rb = kcd::clampi(A.ref_off[b0 + k], 0, A.n_refs);
          const int re = kcd::clampi(A.ref_off[b0 + k + 1], rb, A.n_refs);
          const int rc = min(re - rb, A.max_refs);
          for (int r = 0; r < rc; ++r) {
            const float *rr = A.ref + (int64_t)(rb + r) * dd;
            float dn = 0.f, dx = 0.f;
#pragma unroll
            for (int a = 0; a < DM; ++a) {
              if (a < dd) {
                const float g = fmaxf(fmaxf(rr[a] - thi[a], tlo[a] - rr[a]), 0.f);
                const float u = fmaxf(thi[a] - rr[a], rr[a] - tlo[a]);
                dn = (a == 0) ? g * g : __builtin_fmaf(g, g, dn);
                dx = (a == 0) ? u * u : __builtin_fmaf(u, u, dx);
              }
            }
            far_all = far_all || dn > A.t_alpha;
            far_none = far_none && !(dx > A.t_alpha);
          }
        }
        ub_all = far_all;
        ub_none = in_all && far_none;
      }
    }
  }
  // node-wide values: minimum over the node's lanes; AND / OR of the flags
  alo = kcd::group_min(alo, KP);
  ahi = kcd::group_min(ahi, KP);
  const uint64_t seg = KP >= 64 ? ~0ull : ((1ull << KP) - 1ull);
  const uint64_t b_nall = __ballot(!ub_all), b_none = __ballot(ub_none);
  const int sh = jn << lg;
  const bool uba = ((b_nall >> sh) & seg) == 0, ubn = ((b_none >> sh) & seg) != 0;
  keep_all = __ballot(k == 0 && node_ok && (!(alo < A.t_beta) || ubn));
  red_all = __ballot(k == 0 && (!node_ok || (ahi < A.t_beta && uba)));
}

// Each lane holds PER consecutive samples, so a wavefront's tile is 64 * PER
// consecutive samples (coherent when the samples are spatially ordered). A
// sample is redundant when it is redundant in every open node; the node loop
// stops once no lane's sample can still be. TS: tile decisions settle a node
// for the whole tile where they can (the per-sample test runs only for the
// nodes they leave open); the flags are the same either way.
template <int D, bool TS>
__global__ __launch_bounds__(WG) void k_reduce_flags(FlagArgs A) {
  constexpr int DM = D ? D : 16;
  constexpr int PER = per_lane(D), TILE = WG * PER;
  const int dd = D ? D : A.d;
  __shared__ uint32_t s_cnt[WG / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t s0 = (int64_t)blockIdx.x * TILE + (int64_t)tid * PER;
  float xv[PER][DM];
  bool valid[PER], red[PER];
#pragma unroll
  for (int a = 0; a < DM; ++a) {
    const float *p = A.x + (int64_t)a * A.ld + s0;
    if (a < dd && s0 + PER <= A.n && ((uintptr_t)p & 15) == 0) {
#pragma unroll
      for (int q = 0; q < PER / 4; ++q) {
        const float4 v = reinterpret_cast<const float4 *>(p)[q];
        xv[4 * q][a] = v.x;
        xv[4 * q + 1][a] = v.y;
        xv[4 * q + 2][a] = v.z;
        xv[4 * q + 3][a] = v.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < PER; ++j) xv[j][a] = (a < dd && s0 + j < A.n) ? p[j] : 0.f;
    }
  }
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    valid[j] = s0 + j < A.n;
    red[j] = valid[j];  // redundant everywhere until a node shows otherwise
  }
  auto any_red = [&]() {
    bool r = false;
#pragma unroll
    for (int j = 0; j < PER; ++j) r = r || red[j];
    return __ballot(r) != 0;
  };
  float tlo[DM], thi[DM];
  if constexpr (TS) {
#pragma unroll
    for (int a = 0; a < DM; ++a) {
      float l = INFINITY, h = -INFINITY;
      if (a < dd) {
#pragma unroll
        for (int j = 0; j < PER; ++j)
          if (valid[j]) {
            l = fminf(l, xv[j][a]);
            h = fmaxf(h, xv[j][a]);
          }
      }
      tlo[a] = __int_as_float(__builtin_amdgcn_readfirstlane(
          __float_as_int(kcd::fdec(kcd::wave_min_u32(kcd::ford(l))))));
      thi[a] = __int_as_float(__builtin_amdgcn_readfirstlane(
          __float_as_int(kcd::fdec(kcd::wave_max_u32(kcd::ford(h))))));
    }
  }
  const int lg = A.lg_kp;
  const int npg = TS ? (64 >> lg) : A.n_nodes;
  for (int g0 = 0; g0 < A.n_nodes; g0 += npg) {
    if (!any_red()) break;
    uint64_t keep_all = 0, red_all = 0;
    if constexpr (TS) {
      classify_nodes<DM>(A, g0, lg, tlo, thi, dd, lane, keep_all, red_all);
      if (keep_all) {  // some node keeps every sample of the tile
#pragma unroll
        for (int j = 0; j < PER; ++j) red[j] = false;
        break;
      }
    }
    const int g1 = min(A.n_nodes, g0 + npg);
    for (int m = g0; m < g1; ++m) {
      if (TS && ((red_all >> ((m - g0) << lg)) & 1ull)) continue;
      if (!any_red()) break;
#pragma unroll
      for (int j = 0; j < PER; ++j)
        if (red[j]) red[j] = redundant_in_node<D>(A, m, xv[j], dd);
    }
  }
  uint32_t kept = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const bool keep = valid[j] && !red[j];
    if (valid[j]) A.keep[s0 + j] = keep ? 1 : 0;
    kept += keep;
  }
  const uint32_t w = kcd::wave_sum_u32(kept);
  if (lane == 0) s_cnt[wave] = w;
  __syncthreads();
  if (tid == 0) {
    uint32_t t = 0;
    for (int i = 0; i < WG / 64; ++i) t += s_cnt[i];
    A.tile_cnt[blockIdx.x] = t;
  }
}

// Tile offsets in two levels: k_scan_local scans SCAN_BLOCK tile counts per
// workgroup (block-local exclusive offsets, at most 2^23, and the block's
// total); k_reduce_scan then scans the block totals in one workgroup. A
// tile's output position is its block's offset plus its local offset.
constexpr int SCAN_PER = 8;
constexpr int SCAN_BLOCK = WG * SCAN_PER;

__global__ __launch_bounds__(WG) void k_scan_local(const uint32_t *cnt, int64_t n_tiles,
                                                   uint32_t *off, uint32_t *bsum) {
  __shared__ uint32_t s_w[WG / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * SCAN_BLOCK + (int64_t)tid * SCAN_PER;
  uint32_t v[SCAN_PER], sum = 0;
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) {
    v[j] = i0 + j < n_tiles ? cnt[i0 + j] : 0u;
    sum += v[j];
  }
  uint32_t x = sum;  // inclusive scan over the wavefront
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_w[wave] = x;
  __syncthreads();
  uint32_t wbase = 0;
  for (int w = 0; w < wave; ++w) wbase += s_w[w];
  uint32_t run = wbase + x - sum;
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) {
    if (i0 + j < n_tiles) off[i0 + j] = run;
    run += v[j];
  }
  if (tid == WG - 1) bsum[blockIdx.x] = wbase + x;
}

// One workgroup: exclusive scan of the block totals; total into *n_out.
__global__ __launch_bounds__(1024) void k_reduce_scan(const uint32_t *cnt, int64_t n_tiles,
                                                      int64_t *off, int64_t *n_out) {
  __shared__ int64_t s[1024];
  const int t = threadIdx.x;
  const int64_t per = (n_tiles + 1023) / 1024;
  const int64_t a = (int64_t)t * per;
  const int64_t b = a + per < n_tiles ? a + per : n_tiles;
  int64_t sum = 0;
  for (int64_t i = a; i < b; ++i) sum += cnt[i];
  s[t] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int64_t v = t >= o ? s[t - o] : 0;
    __syncthreads();
    s[t] += v;
    __syncthreads();
  }
  int64_t run = s[t] - sum;  // exclusive prefix of this thread's chunk
  for (int64_t i = a; i < b; ++i) {
    off[i] = run;
    run += cnt[i];
  }
  if (t == 1023) *n_out = s[1023];
}

template <int D>
__global__ __launch_bounds__(WG) void k_reduce_scatter(const float *x, int64_t n, int64_t ld,
                                                       int d, const uint32_t *idx_in,
                                                       const uint8_t *keep, const uint32_t *off,
                                                       const int64_t *boff,
                                                       float *x_out, uint32_t *idx_out,
                                                       int64_t ld_out) {
  constexpr int DM = D ? D : 16;
  constexpr int PER = per_lane(D), TILE = WG * PER;
  const int dd = D ? D : d;
  __shared__ uint32_t s_w[PER][WG / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t base = (int64_t)blockIdx.x * TILE;
  bool kp[PER];
  uint64_t bal[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int64_t s = base + (int64_t)j * WG + tid;
    kp[j] = s < n && keep[s] != 0;
    bal[j] = __ballot(kp[j]);
    if (lane == 0) s_w[j][wave] = (uint32_t)__popcll(bal[j]);
  }
  __syncthreads();
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  int64_t pos0 = boff[blockIdx.x / SCAN_BLOCK] + off[blockIdx.x];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    // samples are ordered (j, wave, lane) within the tile
    int64_t p = pos0;
    for (int w = 0; w < wave; ++w) p += s_w[j][w];
    p += __popcll(bal[j] & below);
    const int64_t s = base + (int64_t)j * WG + tid;
    if (kp[j]) {
#pragma unroll
      for (int a = 0; a < DM; ++a)
        if (a < dd) x_out[(int64_t)a * ld_out + p] = x[(int64_t)a * ld + s];
      idx_out[p] = idx_in ? idx_in[s] : (uint32_t)s;
    }
    for (int w = 0; w < WG / 64; ++w) pos0 += s_w[j][w];
  }
}

#define KCR_D(DV)                                                          \
  case DV:                                                                 \
    if (flags && skip)                                                     \
      k_reduce_flags<DV, true><<<grid, WG, 0, st>>>(*FA);                  \
    else if (flags)                                                        \
      k_reduce_flags<DV, false><<<grid, WG, 0, st>>>(*FA);                 \
    else                                                                   \
      k_reduce_scatter<DV><<<grid, WG, 0, st>>>(SA.x, SA.n, SA.ld, SA.d, SA.idx_in, SA.keep, \
                                                SA.off, SA.boff, SA.x_out, SA.idx_out,        \
                                                SA.ld_out);                                   \
    return KC_OK;

struct ScatterArgs {
  const float *x;
  int64_t n, ld;
  int d;
  const uint32_t *idx_in;
  const uint8_t *keep;
  const uint32_t *off;
  const int64_t *boff;
  float *x_out;
  uint32_t *idx_out;
  int64_t ld_out;
};

static kc_status launch(int d, bool flags, bool skip, const FlagArgs *FA, const ScatterArgs &SA,
                        int64_t grid, hipStream_t st) {
  switch (d <= 8 ? d : 0) {
    KCR_D(1)
    KCR_D(2)
    KCR_D(3)
    KCR_D(4)
    KCR_D(5)
    KCR_D(6)
    KCR_D(7)
    KCR_D(8)
    KCR_D(0)
  }
  return KC_EUNSUPPORTED;
}

}  // namespace kcr

using namespace kcr;

// Tile decisions on unless the autotune table holds "r_d<d>" with skip 0
// (tests compare the two paths).
static bool reduce_tiles(kc_handle *h, int d) {
  char key[32];
  snprintf(key, sizeof key, "r_d%d", d);
  const auto it = h->tune.find(std::string_view(key));
  return it == h->tune.end() || it->second.skip != 0;
}

static kc_status count_impl(kc_handle *h, const kc_points *in, const kc_nodes *open,
                            const kc_refs *refs, double beta, double alpha, uint8_t *keep,
                            int64_t *n_out, hipStream_t st) {
  const int64_t n_tiles = (in->n + tile_of(in->d) - 1) / tile_of(in->d);
  const int64_t n_blocks = (n_tiles + SCAN_BLOCK - 1) / SCAN_BLOCK;
  const size_t keep_bytes = keep ? 0 : (((size_t)in->n + 255) & ~(size_t)255);
  const size_t cnt_bytes = (((size_t)n_tiles * 4) + 255) & ~(size_t)255;
  const size_t off_bytes = (((size_t)n_tiles * 4) + 255) & ~(size_t)255;
  const size_t bsum_bytes = (((size_t)n_blocks * 4) + 255) & ~(size_t)255;
  const size_t boff_bytes = (size_t)n_blocks * 8;
  void *scr = nullptr;
  kc_status s =
      kc_get_scratch(h, keep_bytes + cnt_bytes + off_bytes + bsum_bytes + boff_bytes, &scr);
  if (s != KC_OK) return s;
  uint8_t *kf = keep ? keep : (uint8_t *)scr;
  char *sp = (char *)scr + keep_bytes;
  uint32_t *tcnt = (uint32_t *)sp;
  uint32_t *toff = (uint32_t *)(sp + cnt_bytes);
  uint32_t *bsum = (uint32_t *)(sp + cnt_bytes + off_bytes);
  int64_t *boff = (int64_t *)(sp + cnt_bytes + off_bytes + bsum_bytes);

  FlagArgs A;
  A.x = in->x;
  A.n = in->n;
  A.ld = in->ld;
  A.d = in->d;
  A.n_nodes = open->n_nodes;
  A.n_boxes = open->n_boxes;
  A.k_max = open->k_max;
  A.box_off = open->box_off;
  A.lo = open->lo;
  A.hi = open->hi;
  A.ref_off = refs ? refs->ref_off : nullptr;
  A.ref = refs ? refs->ref : nullptr;
  A.n_refs = refs ? refs->n_refs : 0;
  A.max_refs = refs ? refs->max_per_box : 0;
  A.t_beta = kc_thr_lt(beta, in->d);
  A.t_alpha = kc_thr_gt(alpha, in->d);
  A.keep = kf;
  A.tile_cnt = tcnt;
  ScatterArgs SA{};
  h->red.x = nullptr;
  int lg = 0;
  while ((1 << lg) < open->k_max && lg < 6) ++lg;
  A.lg_kp = lg;
  s = launch(in->d, true, reduce_tiles(h, in->d), &A, SA, n_tiles, st);
  if (s != KC_OK) return kc_fail(h, s, "reduce flags launch");
  s = kc_check_launch(h, "k_reduce_flags");
  if (s != KC_OK) return s;
  k_scan_local<<<(unsigned)n_blocks, WG, 0, st>>>(tcnt, n_tiles, toff, bsum);
  s = kc_check_launch(h, "k_scan_local");
  if (s != KC_OK) return s;
  k_reduce_scan<<<1, 1024, 0, st>>>(bsum, n_blocks, boff, n_out);
  s = kc_check_launch(h, "k_reduce_scan");
  if (s != KC_OK) return s;
  h->red.x = in->x;
  h->red.n = in->n;
  h->red.scratch = scr;
  h->red.keep_bytes = keep_bytes;
  h->red.cnt_bytes = cnt_bytes;
  h->red.off_bytes = off_bytes;
  h->red.bsum_bytes = bsum_bytes;
  return KC_OK;
}

// Scatter with the flags of the last count over the same points; `keep` is
// the caller's flag array when the count wrote there.
static kc_status compact_impl(kc_handle *h, const kc_points *in, const uint32_t *idx_in,
                              const uint8_t *keep, float *x_out, uint32_t *idx_out, int64_t ld_out,
                              hipStream_t st) {
  KC_RETURN_IF(h->red.x != in->x || h->red.n != in->n || h->red.scratch != h->scratch, h,
               KC_EINVAL, "compaction without a matching count of the same samples");
  const int64_t n_tiles = (in->n + tile_of(in->d) - 1) / tile_of(in->d);
  char *scr = (char *)h->red.scratch;
  const uint8_t *kf = keep ? keep : (const uint8_t *)scr;
  const uint32_t *toff = (const uint32_t *)(scr + h->red.keep_bytes + h->red.cnt_bytes);
  const int64_t *boff = (const int64_t *)(scr + h->red.keep_bytes + h->red.cnt_bytes +
                                          h->red.off_bytes + h->red.bsum_bytes);
  ScatterArgs SA{in->x, in->n, in->ld, in->d, idx_in, kf, toff, boff, x_out, idx_out, ld_out};
  h->red.x = nullptr;
  kc_status s = launch(in->d, false, false, nullptr, SA, n_tiles, st);
  if (s != KC_OK) return kc_fail(h, s, "reduce scatter launch");
  return kc_check_launch(h, "k_reduce_scatter");
}

kc_status kc_reduce_count(kc_handle *h, const kc_points *in, const kc_nodes *open,
                          const kc_refs *refs, double beta, double alpha, int64_t *n_out,
                          hipStream_t st) {
  kc_status s = kc_validate_points(h, in);
  if (s != KC_OK) return s;
  s = kc_validate_nodes(h, open, in);
  if (s != KC_OK) return s;
  s = kc_validate_refs(h, refs, open);
  if (s != KC_OK) return s;
  KC_RETURN_IF(!n_out, h, KC_EINVAL, "n_out is NULL");
  KC_RETURN_IF(std::isnan(beta) || std::isnan(alpha), h, KC_EINVAL, "beta / alpha is NaN");
  return count_impl(h, in, open, refs, beta, alpha, nullptr, n_out, st);
}

kc_status kc_reduce_compact(kc_handle *h, const kc_points *in, const uint32_t *idx_in,
                            int64_t n_keep, float *x_out, uint32_t *idx_out, int64_t ld_out,
                            hipStream_t st) {
  KC_RETURN_IF(!x_out || !idx_out, h, KC_EINVAL, "x_out / idx_out is NULL");
  KC_RETURN_IF(n_keep < 0 || n_keep > in->n || ld_out < n_keep, h, KC_EINVAL,
               "compaction sizes (n_keep %lld, ld_out %lld)", (long long)n_keep,
               (long long)ld_out);
  return compact_impl(h, in, idx_in, nullptr, x_out, idx_out, ld_out, st);
}

extern "C" kc_status kc_reduce(kc_handle *h, const kc_points *in, const uint32_t *idx_in,
                               const kc_nodes *open, const kc_refs *refs, double beta,
                               double alpha, uint8_t *keep, float *x_out, uint32_t *idx_out,
                               int64_t ld_out, int64_t *n_out, void *stream) {
  return kc_guard(h, [&]() -> kc_status {
    if (!h) return KC_EINVAL;
    kc_status s = kc_validate_points(h, in);
    if (s != KC_OK) return s;
    s = kc_validate_nodes(h, open, in);
    if (s != KC_OK) return s;
    s = kc_validate_refs(h, refs, open);
    if (s != KC_OK) return s;
    KC_RETURN_IF(!x_out || !idx_out || !n_out, h, KC_EINVAL, "x_out / idx_out / n_out is NULL");
    KC_RETURN_IF(ld_out < in->n, h, KC_EINVAL, "ld_out < n");
    KC_RETURN_IF(std::isnan(beta) || std::isnan(alpha), h, KC_EINVAL, "beta / alpha is NaN");
    hipStream_t st = (hipStream_t)stream;
    s = count_impl(h, in, open, refs, beta, alpha, keep, n_out, st);
    if (s != KC_OK) return s;
    return compact_impl(h, in, idx_in, keep, x_out, idx_out, ld_out, st);
  });
}
