// kc_tighten.hip -- cluster assignment and bounds-tightening aggregates
// (Algorithms 3 and 4, Section 4.1) for a batch of nodes in one pass.
//
// A workgroup owns one node, a chunk of KC of its boxes and one split of the
// samples. Every lane evaluates, for its samples, beta_s^k against all boxes of
// the node (center-based assignment), the distances to the refs (sample-based
// assignment and the balls of S_+^k), and folds the samples into per-box
// running min / max / count registers for the boxes of its chunk. Wavefront
// shuffles and one integer atomic per value and wavefront finish the
// reduction; floats travel as order-preserving integers, so the result does not
// depend on the order of the atomics.
#include <cmath>

#include "kc_device.h"
#include "kc_internal.h"

namespace kct {

constexpr int WG = 256;

struct TightenArgs {
  const float *x;
  int64_t n, ld;
  int d;
  int n_nodes, n_boxes, k_max;
  const int32_t *box_off;
  const float *lo, *hi;
  const int32_t *ref_off;  // null: no refs
  const float *ref;
  int n_refs, max_refs;
  float t_center;  // beta > t_center   => excluded from the box's cluster
  float t_sample;  // dist > t_sample    => not with that ref (4 alpha)
  float t_ball;    // dist <= t_ball     => inside the ball of the ref (alpha)
  int n_chunks, kc;
  int64_t span;
  uint32_t *bb_lo, *bb_hi, *asg_min, *asg_max;  // order-preserving encodings
  uint32_t *n_in, *n_asg, *n_excl;
  int8_t *labels;
};

template <int D, int KC>
__global__ __launch_bounds__(WG) void k_tighten(TightenArgs A) {
  constexpr int DM = D ? D : 16;
  const int dd = D ? D : A.d;
  extern __shared__ float sm[];  // boxes [k_max][2*DM] then refs [*][DM]
  __shared__ int s_b0, s_cnt, s_allref, s_r0, s_rtot;
  __shared__ int s_rbeg[64], s_rcnt[64];

  const int tid = threadIdx.x, lane = tid & 63;
  const int u = kcd::xcd_unit(blockIdx.x, gridDim.x);
  const int chunk = u % A.n_chunks;
  const int rest = u / A.n_chunks;
  const int m = rest % A.n_nodes, split = rest / A.n_nodes;

  if (tid == 0) {
    const int b0 = kcd::clampi(A.box_off[m], 0, A.n_boxes);
    const int b1 = kcd::clampi(A.box_off[m + 1], b0, A.n_boxes);
    const int cnt = min(b1 - b0, A.k_max);
    s_b0 = b0;
    s_cnt = cnt;
    int all = cnt > 0 && A.ref_off != nullptr;
    int r0 = 0, tot = 0;
    if (A.ref_off) r0 = kcd::clampi(A.ref_off[b0], 0, A.n_refs);
    for (int k = 0; k < cnt; ++k) {
      int rb = 0, rc = 0;
      if (A.ref_off) {
        rb = kcd::clampi(A.ref_off[b0 + k], 0, A.n_refs);
        const int re = kcd::clampi(A.ref_off[b0 + k + 1], rb, A.n_refs);
        rc = min(re - rb, A.max_refs);
      }
      s_rbeg[k] = tot;  // position in the LDS copy
      s_rcnt[k] = rc;
      s_rcnt[k] = rc;
      tot += rc;
      if (rc == 0) all = 0;
      (void)rb;
    }
    s_r0 = r0;
    s_rtot = tot;
    s_allref = all;
  }
  __syncthreads();
  const int cnt = s_cnt;
  float *bx = sm;
  float *rf = sm + A.k_max * 2 * DM;
  for (int i = tid; i < A.k_max * DM; i += WG) {
    const int k = i / DM, a = i - k * DM;
    float l = 0.f, h = 0.f;
    if (k < cnt && a < dd) {
      l = A.lo[(int64_t)(s_b0 + k) * dd + a];
      h = A.hi[(int64_t)(s_b0 + k) * dd + a];
    }
    bx[k * 2 * DM + 2 * a] = l;
    bx[k * 2 * DM + 2 * a + 1] = h;
  }
  if (A.ref_off) {
    // refs of box k are copied densely in box order
    for (int k = 0; k < cnt; ++k) {
      const int rb = kcd::clampi(A.ref_off[s_b0 + k], 0, A.n_refs);
      for (int i = tid; i < s_rcnt[k] * DM; i += WG) {
        const int r = i / DM, a = i - r * DM;
        rf[(s_rbeg[k] + r) * DM + a] = a < dd ? A.ref[(int64_t)(rb + r) * dd + a] : 0.f;
      }
    }
  }
  __syncthreads();

  const int c0 = chunk * A.kc;
  float bmin[KC][DM], bmax[KC][DM], amin[KC][DM], amax[KC][DM];
  uint32_t nin[KC], nasg[KC];
#pragma unroll
  for (int kk = 0; kk < KC; ++kk) {
    nin[kk] = 0;
    nasg[kk] = 0;
#pragma unroll
    for (int a = 0; a < DM; ++a) {
      bmin[kk][a] = INFINITY;
      bmax[kk][a] = -INFINITY;
      amin[kk][a] = INFINITY;
      amax[kk][a] = -INFINITY;
    }
  }
  uint32_t nex = 0;
  const bool allref = s_allref != 0;
  const bool write_labels = A.labels != nullptr && chunk == 0;

  const int64_t s_lo = (int64_t)split * A.span;
  const int64_t s_hi = min(A.n, s_lo + A.span);
  for (int64_t s = s_lo + tid; s < s_hi; s += WG) {
    float xv[DM];
#pragma unroll
    for (int a = 0; a < DM; ++a) xv[a] = a < dd ? A.x[(int64_t)a * A.ld + s] : 0.f;

    // Center-based assignment (Lemma 1).
    int n_out = 0, keep = -1;
    for (int k = 0; k < cnt; ++k) {
      float acc = 0.f;
#pragma unroll
      for (int a = 0; a < DM; ++a) {
        if (a < dd) {
          const float c = kcd::med3(bx[k * 2 * DM + 2 * a], xv[a], bx[k * 2 * DM + 2 * a + 1]);
          const float t = xv[a] - c;
          acc = (a == 0) ? t * t : __builtin_fmaf(t, t, acc);
        }
      }
      if (acc > A.t_center)
        ++n_out;
      else
        keep = k;
    }
    int label = -1;
    if (n_out == cnt)
      label = -2;
    else if (n_out == cnt - 1)
      label = keep;

    // Sample-based assignment (Lemma 2), only for unassigned samples.
    if (label == -1 && allref) {
      int n_far = 0, rest_k = -1;
      for (int k = 0; k < cnt; ++k) {
        bool far = false;
        for (int r = 0; r < s_rcnt[k]; ++r) {
          const float *rr = rf + (s_rbeg[k] + r) * DM;
          float acc = 0.f;
#pragma unroll
          for (int a = 0; a < DM; ++a) {
            if (a < dd) {
              const float t = xv[a] - rr[a];
              acc = (a == 0) ? t * t : __builtin_fmaf(t, t, acc);
            }
          }
          far = far || (acc > A.t_sample);
        }
        if (far)
          ++n_far;
        else
          rest_k = k;
      }
      if (n_far == cnt - 1) label = rest_k;
    }
    if (write_labels) A.labels[s] = (int8_t)label;
    nex += (label == -2);

#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const int k = c0 + kk;
      if (k < cnt) {
        if (label == k) {
          ++nasg[kk];
#pragma unroll
          for (int a = 0; a < DM; ++a) {
            amin[kk][a] = fminf(amin[kk][a], xv[a]);
            amax[kk][a] = fmaxf(amax[kk][a], xv[a]);
          }
        }
        // S_+^k: inside box k and within the ball of every ref of box k.
        bool in = true;
#pragma unroll
        for (int a = 0; a < DM; ++a)
          if (a < dd) in = in && (bx[k * 2 * DM + 2 * a] <= xv[a]) && (xv[a] <= bx[k * 2 * DM + 2 * a + 1]);
        if (in) {
          for (int r = 0; r < s_rcnt[k]; ++r) {
            const float *rr = rf + (s_rbeg[k] + r) * DM;
            float acc = 0.f;
#pragma unroll
            for (int a = 0; a < DM; ++a) {
              if (a < dd) {
                const float t = xv[a] - rr[a];
                acc = (a == 0) ? t * t : __builtin_fmaf(t, t, acc);
              }
            }
            in = in && (acc <= A.t_ball);
          }
        }
        if (in) {
          ++nin[kk];
#pragma unroll
          for (int a = 0; a < DM; ++a) {
            bmin[kk][a] = fminf(bmin[kk][a], xv[a]);
            bmax[kk][a] = fmaxf(bmax[kk][a], xv[a]);
          }
        }
      }
    }
  }

  // Wavefront reduction, then one atomic per value and wavefront.
#pragma unroll
  for (int kk = 0; kk < KC; ++kk) {
    const int k = c0 + kk;
    const uint32_t ci = kcd::wave_sum_u32(nin[kk]);
    const uint32_t ca = kcd::wave_sum_u32(nasg[kk]);
    if (k < cnt) {
      const int64_t b = s_b0 + k;
      if (lane == 0 && ci) atomicAdd(&A.n_in[b], ci);
      if (lane == 0 && ca) atomicAdd(&A.n_asg[b], ca);
    }
#pragma unroll
    for (int a = 0; a < DM; ++a) {
      const uint32_t v0 = kcd::wave_min_u32(kcd::ford(bmin[kk][a]));
      const uint32_t v1 = kcd::wave_max_u32(kcd::ford(bmax[kk][a]));
      const uint32_t v2 = kcd::wave_min_u32(kcd::ford(amin[kk][a]));
      const uint32_t v3 = kcd::wave_max_u32(kcd::ford(amax[kk][a]));
      if (k < cnt && a < dd && lane == 0) {
        const int64_t o = (int64_t)(s_b0 + k) * dd + a;
        if (ci) {
          atomicMin(&A.bb_lo[o], v0);
          atomicMax(&A.bb_hi[o], v1);
        }
        if (ca) {
          atomicMin(&A.asg_min[o], v2);
          atomicMax(&A.asg_max[o], v3);
        }
      }
    }
  }
  if (chunk == 0) {
    const uint32_t e = kcd::wave_sum_u32(nex);
    if (lane == 0 && e) atomicAdd(&A.n_excl[m], e);
  }
}

__global__ void k_tighten_init(uint32_t *bb_lo, uint32_t *bb_hi, uint32_t *amn, uint32_t *amx,
                               uint32_t *n_in, uint32_t *n_asg, int64_t nbd, int nb,
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
  }
  if (i < nn) n_excl[i] = 0;
}

__global__ void k_tighten_decode(uint32_t *a, uint32_t *b, uint32_t *c, uint32_t *e, int64_t nbd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nbd) {
    a[i] = __float_as_uint(kcd::fdec(a[i]));
    b[i] = __float_as_uint(kcd::fdec(b[i]));
    c[i] = __float_as_uint(kcd::fdec(c[i]));
    e[i] = __float_as_uint(kcd::fdec(e[i]));
  }
}

#define KCT_CASE(DV, KCV)                                                 \
  if (d == DV && kc == KCV) {                                             \
    k_tighten<(DV <= 8 ? DV : 0), KCV><<<grid, WG, lds, st>>>(A);         \
    return KC_OK;                                                         \
  }
#define KCT_D(DV) KCT_CASE(DV, 1) KCT_CASE(DV, 2) KCT_CASE(DV, 4) KCT_CASE(DV, 8)

static kc_status launch(int d, int kc, const TightenArgs &A, int grid, size_t lds, hipStream_t st) {
  KCT_D(1) KCT_D(2) KCT_D(3) KCT_D(4) KCT_D(5) KCT_D(6) KCT_D(7) KCT_D(8)
  if (d > 8) {
    if (kc == 1) { k_tighten<0, 1><<<grid, WG, lds, st>>>(A); return KC_OK; }
    if (kc == 2) { k_tighten<0, 2><<<grid, WG, lds, st>>>(A); return KC_OK; }
  }
  return KC_EUNSUPPORTED;
}

}  // namespace kct

using namespace kct;

extern "C" kc_status kc_tighten(kc_handle *h, const kc_points *pts, const kc_nodes *nodes,
                                double alpha, const kc_refs *refs, float *bb_lo, float *bb_hi,
                                uint32_t *n_in, float *asg_min, float *asg_max, uint32_t *n_asg,
                                uint32_t *n_excl, int8_t *labels, void *stream) {
  if (!h) return KC_EINVAL;
  kc_status s = kc_validate_points(h, pts);
  if (s != KC_OK) return s;
  s = kc_validate_nodes(h, nodes, pts);
  if (s != KC_OK) return s;
  s = kc_validate_refs(h, refs, nodes);
  if (s != KC_OK) return s;
  KC_RETURN_IF(!bb_lo || !bb_hi || !n_in || !asg_min || !asg_max || !n_asg || !n_excl, h,
               KC_EINVAL, "an output array is NULL");
  KC_RETURN_IF(labels && nodes->n_nodes != 1, h, KC_EINVAL, "labels need n_nodes == 1");
  KC_RETURN_IF(std::isnan(alpha) || alpha < 0, h, KC_EINVAL, "alpha must be >= 0");
  hipStream_t st = (hipStream_t)stream;
  const int d = pts->d, DM = d <= 8 ? d : 16;
  // boxes per chunk: as many as fit in about 112 registers of aggregates
  int kc = 8;
  while (kc > 1 && kc * (4 * DM + 2) > 112) kc /= 2;
  if (d > 8 && kc > 2) kc = 2;
  while (kc > 1 && kc / 2 >= nodes->k_max) kc /= 2;
  const int n_chunks = (nodes->k_max + kc - 1) / kc;
  const int max_refs = refs ? refs->max_per_box : 0;
  const size_t lds = ((size_t)nodes->k_max * 2 * DM + (size_t)nodes->k_max * max_refs * DM) * 4;
  KC_RETURN_IF(lds > h->lds_per_block, h, KC_EUNSUPPORTED, "boxes and refs of a node exceed LDS");
  const int64_t units = (int64_t)nodes->n_nodes * n_chunks;
  const int64_t target = (int64_t)h->n_cu * 8;
  int64_t splits = (target + units - 1) / units;
  int64_t span = (pts->n + splits - 1) / splits;
  span = (span + WG - 1) / WG * WG;
  splits = (pts->n + span - 1) / span;
  const int64_t grid = splits * units;
  KC_RETURN_IF(grid > 0x7fffffff, h, KC_EUNSUPPORTED, "grid too large");

  const int64_t nbd = (int64_t)nodes->n_boxes * d;
  const int64_t ni = nbd > nodes->n_boxes ? nbd : nodes->n_boxes;
  const int64_t nmax = ni > nodes->n_nodes ? ni : nodes->n_nodes;
  if (nmax > 0)
    k_tighten_init<<<(nmax + 255) / 256, 256, 0, st>>>(
        (uint32_t *)bb_lo, (uint32_t *)bb_hi, (uint32_t *)asg_min, (uint32_t *)asg_max, n_in,
        n_asg, nbd, nodes->n_boxes, n_excl, nodes->n_nodes);
  s = kc_check_launch(h, "k_tighten_init");
  if (s != KC_OK) return s;

  TightenArgs A;
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
  A.span = span;
  A.bb_lo = (uint32_t *)bb_lo;
  A.bb_hi = (uint32_t *)bb_hi;
  A.asg_min = (uint32_t *)asg_min;
  A.asg_max = (uint32_t *)asg_max;
  A.n_in = n_in;
  A.n_asg = n_asg;
  A.n_excl = n_excl;
  A.labels = labels;
  s = launch(d, kc, A, (int)grid, lds, st);
  KC_RETURN_IF(s != KC_OK, h, s, "no tighten variant for d=%d kc=%d", d, kc);
  s = kc_check_launch(h, "k_tighten");
  if (s != KC_OK) return s;
  if (nbd > 0)
    k_tighten_decode<<<(nbd + 255) / 256, 256, 0, st>>>((uint32_t *)bb_lo, (uint32_t *)bb_hi,
                                                        (uint32_t *)asg_min,
                                                        (uint32_t *)asg_max, nbd);
  return kc_check_launch(h, "k_tighten_decode");
}
