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
  uint64_t *asg_far;  // per box: max key (dist to midpoint, ~index); may be null
  int8_t *labels;
};

__device__ __forceinline__ float sqdist(const float *xv, const float *r, int dd, int DM) {
  float acc = 0.f;
  for (int a = 0; a < DM; ++a) {
    if (a < dd) {
      const float t = xv[a] - r[a];
      acc = (a == 0) ? t * t : __builtin_fmaf(t, t, acc);
    }
  }
  return acc;
}

// Squared distances from x to the nearest point and to the farthest corner of
// the box [b[2a], b[2a+1]], in the same operation order as sqdist. Rounding is
// monotone, so for every point r of the box the computed sqdist(x, r) lies
// between the two: a threshold test that the bounding box of a set of refs
// settles gives the same answer as testing each ref.
__device__ __forceinline__ float box_near(const float *xv, const float *b, int dd, int DM) {
  float acc = 0.f;
  for (int a = 0; a < DM; ++a) {
    if (a < dd) {
      const float t = xv[a] - kcd::med3(b[2 * a], xv[a], b[2 * a + 1]);
      acc = (a == 0) ? t * t : __builtin_fmaf(t, t, acc);
    }
  }
  return acc;
}
__device__ __forceinline__ float box_far(const float *xv, const float *b, int dd, int DM) {
  float acc = 0.f;
  for (int a = 0; a < DM; ++a) {
    if (a < dd) {
      const float t = fmaxf(xv[a] - b[2 * a], b[2 * a + 1] - xv[a]);
      acc = (a == 0) ? t * t : __builtin_fmaf(t, t, acc);
    }
  }
  return acc;
}

// True when every one of the `cnt` refs at r lies within squared distance t of
// x. The refs' bounding box settles most samples; the scan stops at the first
// ref farther than t (refs extreme in some attribute come first).
__device__ __forceinline__ bool all_refs_within(const float *xv, const float *rbox, const float *r,
                                                int cnt, float t, int dd, int DM) {
  if (box_near(xv, rbox, dd, DM) > t) return false;
  if (box_far(xv, rbox, dd, DM) <= t) return true;
  for (int i = 0; i < cnt; ++i)
    if (sqdist(xv, r + i * DM, dd, DM) > t) return false;
  return true;
}

// S samples per lane per tile (16-byte loads when S = 4), KC boxes per chunk
// with their aggregates in registers. With all boxes of the node in one chunk
// the box distances of the center-based test also give the inside flags.
// Small shapes (D * KC <= 6) hold few aggregates: ask for six wavefronts per
// SIMD (at most 80 VGPRs) so that memory latency stays hidden.
constexpr int tighten_min_waves(int D, int KC) { return D > 0 && D * KC <= 6 ? 6 : 1; }

// REFS: the node batch carries refs (sample-based assignment and the balls of
// S_+^k); without refs none of that code is compiled in.
template <int D, int KC, int S, bool REFS>
__global__ __launch_bounds__(WG, tighten_min_waves(D, KC)) void k_tighten(TightenArgs A) {
  constexpr int DM = D ? D : 16;
  const int dd = D ? D : A.d;
  extern __shared__ float sm[];  // boxes [k_max][2*DM] then refs [*][DM]
  __shared__ int s_b0, s_cnt, s_allref;
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
    int tot = 0;
    for (int k = 0; k < cnt; ++k) {
      int rc = 0;
      if (A.ref_off) {
        const int rb = kcd::clampi(A.ref_off[b0 + k], 0, A.n_refs);
        const int re = kcd::clampi(A.ref_off[b0 + k + 1], rb, A.n_refs);
        rc = min(re - rb, A.max_refs);
      }
      s_rbeg[k] = tot;  // position in the LDS copy
      s_rcnt[k] = rc;
      tot += rc;
      if (rc == 0) all = 0;
    }
    s_allref = all;
  }
  __syncthreads();
  const int cnt = s_cnt;
  float *bx = sm;
  float *rbx = sm + A.k_max * 2 * DM;  // bounding boxes of each box's refs
  float *rf = rbx + A.k_max * 2 * DM;
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
  if (REFS && A.ref_off) {
    // refs of box k are copied densely in box order
    for (int k = 0; k < cnt; ++k) {
      const int rb = kcd::clampi(A.ref_off[s_b0 + k], 0, A.n_refs);
      for (int i = tid; i < s_rcnt[k] * DM; i += WG) {
        const int r = i / DM, a = i - r * DM;
        rf[(s_rbeg[k] + r) * DM + a] = a < dd ? A.ref[(int64_t)(rb + r) * dd + a] : 0.f;
      }
    }
  }
  if (REFS) {
    __syncthreads();
    // one lane per box: bounding box of its refs, then the refs holding the
    // smallest or largest value of some attribute moved to the front
    if (tid < cnt) {
      float *R = rf + s_rbeg[tid] * DM;
      float *B = rbx + tid * 2 * DM;
      const int rc = s_rcnt[tid];
      for (int a = 0; a < DM; ++a) {
        float l = INFINITY, h = -INFINITY;
        for (int r = 0; r < rc; ++r) {
          l = fminf(l, R[r * DM + a]);
          h = fmaxf(h, R[r * DM + a]);
        }
        B[2 * a] = l;
        B[2 * a + 1] = h;
      }
      int front = 0;
      for (int a = 0; a < dd && front < rc; ++a)
        for (int side = 0; side < 2 && front < rc; ++side) {
          const float ext = side == 0 ? B[2 * a] : B[2 * a + 1];
          bool have = false;  // an earlier front ref already holds the extreme
          for (int r = 0; r < front; ++r) have = have || R[r * DM + a] == ext;
          if (have) continue;
          int best = front;
          while (best < rc && R[best * DM + a] != ext) ++best;
          if (best == rc) continue;
          for (int q = 0; q < DM; ++q) {
            const float t = R[front * DM + q];
            R[front * DM + q] = R[best * DM + q];
            R[best * DM + q] = t;
          }
          ++front;
        }
    }
  }
  __syncthreads();

  const int c0 = chunk * A.kc;
  const bool single = A.n_chunks == 1;
  float bmin[KC][DM], bmax[KC][DM], amin[KC][DM], amax[KC][DM];
  uint32_t nin[KC], nasg[KC];
  uint64_t far[KC];
#pragma unroll
  for (int kk = 0; kk < KC; ++kk) {
    nin[kk] = 0;
    nasg[kk] = 0;
    far[kk] = 0;
#pragma unroll
    for (int a = 0; a < DM; ++a) {
      bmin[kk][a] = INFINITY;
      bmax[kk][a] = -INFINITY;
      amin[kk][a] = INFINITY;
      amax[kk][a] = -INFINITY;
    }
  }
  uint32_t nex = 0;
  const int cnt_u = __builtin_amdgcn_readfirstlane(cnt);
  const bool allref = __builtin_amdgcn_readfirstlane(s_allref) != 0;
  const bool write_labels = A.labels != nullptr && chunk == 0;

  const int64_t s_lo = (int64_t)split * A.span;
  const int64_t s_hi = min(A.n, s_lo + A.span);
  for (int64_t base = s_lo + (int64_t)tid * S; base < s_hi; base += (int64_t)WG * S) {
    float xs[S][DM];
    const bool full = base + S <= s_hi;
#pragma unroll
    for (int a = 0; a < DM; ++a) {
      if (a < dd) {
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
      } else {
#pragma unroll
        for (int i = 0; i < S; ++i) xs[i][a] = 0.f;
      }
    }
    // Center-based assignment (Lemma 1), box-major: each box's bounds are
    // read from LDS once for the lane's S samples. In the single-chunk case
    // the same distances record which boxes hold each sample.
    int n_out[S], keep[S], label[S];
    uint32_t inm[S];
#pragma unroll
    for (int i = 0; i < S; ++i) {
      n_out[i] = 0;
      keep[i] = -1;
      inm[i] = 0;
    }
    if (single) {
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        if (k < cnt_u) {
          float lo[DM], hi[DM];
#pragma unroll
          for (int a = 0; a < DM; ++a) {
            lo[a] = bx[k * 2 * DM + 2 * a];
            hi[a] = bx[k * 2 * DM + 2 * a + 1];
          }
#pragma unroll
          for (int i = 0; i < S; ++i) {
            float acc = 0.f;
            bool in = true;
#pragma unroll
            for (int a = 0; a < DM; ++a) {
              if (a < dd) {
                const float c = kcd::med3(lo[a], xs[i][a], hi[a]);
                in = in && (c == xs[i][a]);
                const float t = xs[i][a] - c;
                acc = (a == 0) ? t * t : __builtin_fmaf(t, t, acc);
              }
            }
            const bool out = acc > A.t_center;
            n_out[i] += out;
            keep[i] = out ? keep[i] : k;
            inm[i] |= (uint32_t)in << k;
          }
        }
      }
    } else {
      for (int k = 0; k < cnt_u; ++k) {
        float lo[DM], hi[DM];
#pragma unroll
        for (int a = 0; a < DM; ++a) {
          lo[a] = bx[k * 2 * DM + 2 * a];
          hi[a] = bx[k * 2 * DM + 2 * a + 1];
        }
#pragma unroll
        for (int i = 0; i < S; ++i) {
          float acc = 0.f;
#pragma unroll
          for (int a = 0; a < DM; ++a) {
            if (a < dd) {
              const float t = xs[i][a] - kcd::med3(lo[a], xs[i][a], hi[a]);
              acc = (a == 0) ? t * t : __builtin_fmaf(t, t, acc);
            }
          }
          const bool out = acc > A.t_center;
          n_out[i] += out;
          keep[i] = out ? keep[i] : k;
        }
      }
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) {
        const int k = c0 + kk;
        if (k < cnt_u) {
#pragma unroll
          for (int i = 0; i < S; ++i) {
            bool in = true;
#pragma unroll
            for (int a = 0; a < DM; ++a)
              if (a < dd)
                in = in && (bx[k * 2 * DM + 2 * a] <= xs[i][a]) && (xs[i][a] <= bx[k * 2 * DM + 2 * a + 1]);
            inm[i] |= (uint32_t)in << kk;
          }
        }
      }
    }

#pragma unroll
    for (int i = 0; i < S; ++i) {
      const float *xv = xs[i];
      int lab = n_out[i] == cnt_u ? -2 : (n_out[i] == cnt_u - 1 ? keep[i] : -1);
      if (base + i >= s_hi) {  // past the end: no contribution
        lab = -3;
        inm[i] = 0;
      }
      // Sample-based assignment (Lemma 2), only for unassigned samples:
      // cluster k is excluded once one of its refs is farther than 4 alpha;
      // the scan stops when two clusters remain possible.
      if (REFS && lab == -1 && allref) {
        int n_near = 0, rest_k = -1;
        for (int k = 0; k < cnt_u && n_near < 2; ++k) {
          const int rb = __builtin_amdgcn_readfirstlane(s_rbeg[k]);
          const int rc = __builtin_amdgcn_readfirstlane(s_rcnt[k]);
          if (all_refs_within(xv, rbx + k * 2 * DM, rf + rb * DM, rc, A.t_sample, dd, DM)) {
            ++n_near;
            rest_k = k;
          }
        }
        if (n_near == 1) lab = rest_k;
      }
      if (write_labels && base + i < s_hi) A.labels[base + i] = (int8_t)lab;
      nex += (lab == -2);
      label[i] = lab;
    }

    // Running aggregates of the chunk's boxes, box-major.
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const int k = c0 + kk;
      if (k < cnt_u) {
        float mid[DM];
#pragma unroll
        for (int a = 0; a < DM; ++a) mid[a] = 0.5f * (bx[k * 2 * DM + 2 * a] + bx[k * 2 * DM + 2 * a + 1]);
        const int rb = __builtin_amdgcn_readfirstlane(s_rbeg[k]);
        const int rc = __builtin_amdgcn_readfirstlane(s_rcnt[k]);
#pragma unroll
        for (int i = 0; i < S; ++i) {
          const float *xv = xs[i];
          if (label[i] == k) {
            ++nasg[kk];
            float dm = 0.f;
#pragma unroll
            for (int a = 0; a < DM; ++a) {
              amin[kk][a] = fminf(amin[kk][a], xv[a]);
              amax[kk][a] = fmaxf(amax[kk][a], xv[a]);
              const float w = xv[a] - mid[a];
              dm = (a == 0) ? w * w : __builtin_fmaf(w, w, dm);
            }
            const uint64_t key = kcd::key_max(dm, (uint32_t)(base + i));
            far[kk] = key > far[kk] ? key : far[kk];
          }
          // S_+^k: inside box k and within the ball of every ref of box k.
          bool in = (inm[i] >> (single ? k : kk)) & 1u;
          if (REFS && in && rc > 0)
            in = all_refs_within(xv, rbx + k * 2 * DM, rf + rb * DM, rc, A.t_ball, dd, DM);
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
  }

  // Wavefront reduction, then one atomic per value and wavefront.
#pragma unroll
  for (int kk = 0; kk < KC; ++kk) {
    const int k = c0 + kk;
    const uint32_t ci = kcd::wave_sum_u32(nin[kk]);
    const uint32_t ca = kcd::wave_sum_u32(nasg[kk]);
    const uint64_t fk = kcd::wave_max_u64(far[kk]);
    if (k < cnt) {
      const int64_t b = s_b0 + k;
      if (lane == 0 && ci) atomicAdd(&A.n_in[b], ci);
      if (lane == 0 && ca) atomicAdd(&A.n_asg[b], ca);
      if (lane == 0 && ca && A.asg_far) atomicMax((unsigned long long *)&A.asg_far[b], (unsigned long long)fk);
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

// samples per lane: 16-byte loads for up to 4 attributes, 8-byte beyond
#define KCT_S(DV) ((DV) > 0 && (DV) <= 4 ? 4 : 2)
#define KCT_CASE(DV, KCV)                                                      \
  if (d == DV && kc == KCV) {                                                  \
    if (refs)                                                                  \
      k_tighten<DV, KCV, KCT_S(DV), true><<<grid, WG, lds, st>>>(A);           \
    else                                                                       \
      k_tighten<DV, KCV, KCT_S(DV), false><<<grid, WG, lds, st>>>(A);          \
    return KC_OK;                                                              \
  }
#define KCT_D(DV) \
  KCT_CASE(DV, 1) KCT_CASE(DV, 2) KCT_CASE(DV, 3) KCT_CASE(DV, 4) KCT_CASE(DV, 5) KCT_CASE(DV, 6) KCT_CASE(DV, 8)

static const int kKC[] = {1, 2, 3, 4, 5, 6, 8};

static kc_status launch(int d, int kc, bool refs, const TightenArgs &A, int grid, size_t lds,
                        hipStream_t st) {
  KCT_D(1) KCT_D(2) KCT_D(3) KCT_D(4) KCT_D(5) KCT_D(6) KCT_D(7) KCT_D(8)
  if (d > 8) {
    if (kc == 1) {
      if (refs) k_tighten<0, 1, 2, true><<<grid, WG, lds, st>>>(A);
      else k_tighten<0, 1, 2, false><<<grid, WG, lds, st>>>(A);
      return KC_OK;
    }
    if (kc == 2) {
      if (refs) k_tighten<0, 2, 2, true><<<grid, WG, lds, st>>>(A);
      else k_tighten<0, 2, 2, false><<<grid, WG, lds, st>>>(A);
      return KC_OK;
    }
  }
  return KC_EUNSUPPORTED;
}

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

}  // namespace kct

using namespace kct;

extern "C" kc_status kc_tighten(kc_handle *h, const kc_points *pts, const kc_nodes *nodes,
                                double alpha, const kc_refs *refs, float *bb_lo, float *bb_hi,
                                uint32_t *n_in, float *asg_min, float *asg_max, uint32_t *n_asg,
                                uint32_t *n_excl, int64_t *asg_far, int8_t *labels, void *stream) {
  return kc_guard(h, [&]() -> kc_status {
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
    const int kc = choose_kc(d, nodes->k_max);
    const int n_chunks = (nodes->k_max + kc - 1) / kc;
    const int max_refs = refs ? refs->max_per_box : 0;
    const size_t lds = ((size_t)nodes->k_max * 4 * DM + (size_t)nodes->k_max * max_refs * DM) * 4;
    KC_RETURN_IF(lds > h->lds_per_block, h, KC_EUNSUPPORTED, "boxes and refs of a node exceed LDS");
    const int S = (d <= 4) ? 4 : 2;
    const int64_t units = (int64_t)nodes->n_nodes * n_chunks;
    const int64_t target = (int64_t)h->n_cu * 8;
    int64_t splits = (target + units - 1) / units;
    int64_t span = (pts->n + splits - 1) / splits;
    span = (span + WG * S - 1) / (WG * S) * (WG * S);
    splits = (pts->n + span - 1) / span;
    const int64_t grid = splits * units;
    KC_RETURN_IF(grid > 0x7fffffff, h, KC_EUNSUPPORTED, "grid too large");
  
    const int64_t nbd = (int64_t)nodes->n_boxes * d;
    const int64_t ni = nbd > nodes->n_boxes ? nbd : nodes->n_boxes;
    const int64_t nmax = ni > nodes->n_nodes ? ni : nodes->n_nodes;
    if (nmax > 0)
      k_tighten_init<<<(nmax + 255) / 256, 256, 0, st>>>(
          (uint32_t *)bb_lo, (uint32_t *)bb_hi, (uint32_t *)asg_min, (uint32_t *)asg_max, n_in,
          n_asg, (uint64_t *)asg_far, nbd, nodes->n_boxes, n_excl, nodes->n_nodes);
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
    A.asg_far = (uint64_t *)asg_far;
    A.labels = labels;
    s = launch(d, kc, A.ref_off != nullptr, A, (int)grid, lds, st);
    KC_RETURN_IF(s != KC_OK, h, s, "no tighten variant for d=%d kc=%d", d, kc);
    s = kc_check_launch(h, "k_tighten");
    if (s != KC_OK) return s;
    if (nmax > 0)
      k_tighten_decode<<<(nmax + 255) / 256, 256, 0, st>>>((uint32_t *)bb_lo, (uint32_t *)bb_hi,
                                                           (uint32_t *)asg_min, (uint32_t *)asg_max,
                                                           nbd, (uint64_t *)asg_far, nodes->n_boxes);
    return kc_check_launch(h, "k_tighten_decode");
  });
}
