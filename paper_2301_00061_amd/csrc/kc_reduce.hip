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
constexpr int PER = 4;  // samples per lane
constexpr int TILE = WG * PER;

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

template <int D>
__global__ __launch_bounds__(WG) void k_reduce_flags(FlagArgs A) {
  constexpr int DM = D ? D : 16;
  const int dd = D ? D : A.d;
  __shared__ uint32_t s_cnt[WG / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t base = (int64_t)blockIdx.x * TILE;
  uint32_t kept = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int64_t s = base + (int64_t)j * WG + tid;
    const bool valid = s < A.n;
    float xv[DM];
#pragma unroll
    for (int a = 0; a < DM; ++a) xv[a] = (valid && a < dd) ? A.x[(int64_t)a * A.ld + s] : 0.f;
    // redundant everywhere until a node shows otherwise
    bool red = valid;
    for (int m = 0; m < A.n_nodes; ++m) {
      if (__ballot(red) == 0) break;
      if (red) red = redundant_in_node<D>(A, m, xv, dd);
    }
    const bool keep = valid && !red;
    if (valid) A.keep[s] = keep ? 1 : 0;
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

// One workgroup: exclusive scan of the tile counts; total into *n_out.
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
                                                       const uint8_t *keep, const int64_t *off,
                                                       float *x_out, uint32_t *idx_out,
                                                       int64_t ld_out) {
  constexpr int DM = D ? D : 16;
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
  int64_t pos0 = off[blockIdx.x];
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
    if (flags)                                                             \
      k_reduce_flags<DV><<<grid, WG, 0, st>>>(*FA);                        \
    else                                                                   \
      k_reduce_scatter<DV><<<grid, WG, 0, st>>>(SA.x, SA.n, SA.ld, SA.d, SA.idx_in, SA.keep, \
                                                SA.off, SA.x_out, SA.idx_out, SA.ld_out);     \
    return KC_OK;

struct ScatterArgs {
  const float *x;
  int64_t n, ld;
  int d;
  const uint32_t *idx_in;
  const uint8_t *keep;
  const int64_t *off;
  float *x_out;
  uint32_t *idx_out;
  int64_t ld_out;
};

static kc_status launch(int d, bool flags, const FlagArgs *FA, const ScatterArgs &SA, int64_t grid,
                        hipStream_t st) {
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

static kc_status count_impl(kc_handle *h, const kc_points *in, const kc_nodes *open,
                            const kc_refs *refs, double beta, double alpha, uint8_t *keep,
                            int64_t *n_out, hipStream_t st) {
  const int64_t n_tiles = (in->n + TILE - 1) / TILE;
  const size_t keep_bytes = keep ? 0 : (((size_t)in->n + 255) & ~(size_t)255);
  const size_t cnt_bytes = (((size_t)n_tiles * 4) + 255) & ~(size_t)255;
  const size_t off_bytes = (size_t)n_tiles * 8;
  void *scr = nullptr;
  kc_status s = kc_get_scratch(h, keep_bytes + cnt_bytes + off_bytes, &scr);
  if (s != KC_OK) return s;
  uint8_t *kf = keep ? keep : (uint8_t *)scr;
  uint32_t *tcnt = (uint32_t *)((char *)scr + keep_bytes);
  int64_t *toff = (int64_t *)((char *)scr + keep_bytes + cnt_bytes);

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
  s = launch(in->d, true, &A, SA, n_tiles, st);
  if (s != KC_OK) return kc_fail(h, s, "reduce flags launch");
  s = kc_check_launch(h, "k_reduce_flags");
  if (s != KC_OK) return s;
  k_reduce_scan<<<1, 1024, 0, st>>>(tcnt, n_tiles, toff, n_out);
  s = kc_check_launch(h, "k_reduce_scan");
  if (s != KC_OK) return s;
  h->red.x = in->x;
  h->red.n = in->n;
  h->red.scratch = scr;
  h->red.keep_bytes = keep_bytes;
  h->red.cnt_bytes = cnt_bytes;
  return KC_OK;
}

// Scatter with the flags of the last count over the same points; `keep` is
// the caller's flag array when the count wrote there.
static kc_status compact_impl(kc_handle *h, const kc_points *in, const uint32_t *idx_in,
                              const uint8_t *keep, float *x_out, uint32_t *idx_out, int64_t ld_out,
                              hipStream_t st) {
  KC_RETURN_IF(h->red.x != in->x || h->red.n != in->n || h->red.scratch != h->scratch, h,
               KC_EINVAL, "compaction without a matching count of the same samples");
  const int64_t n_tiles = (in->n + TILE - 1) / TILE;
  char *scr = (char *)h->red.scratch;
  const uint8_t *kf = keep ? keep : (const uint8_t *)scr;
  const int64_t *toff = (const int64_t *)(scr + h->red.keep_bytes + h->red.cnt_bytes);
  ScatterArgs SA{in->x, in->n, in->ld, in->d, idx_in, kf, toff, x_out, idx_out, ld_out};
  h->red.x = nullptr;
  kc_status s = launch(in->d, false, nullptr, SA, n_tiles, st);
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
