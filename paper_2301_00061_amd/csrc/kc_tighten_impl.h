// kc_tighten_impl.h -- the tightening kernel (template; instantiated per
// attribute count in kc_tighten_d*.hip): cluster assignment and the
// bounds-tightening aggregates of Algorithms 3 and 4 (Section 4.1) for a batch
// of nodes in one pass over the samples.
//
// A workgroup owns NG consecutive nodes (their boxes and refs staged in LDS)
// and one contiguous split of the samples, or -- for nodes with more boxes
// than fit in registers -- one node, a chunk of KC of its boxes and one split.
// Every lane loads S samples per tile (16-byte loads of each structure-of-
// arrays row when S = 4) and, for each of the NG nodes, evaluates beta_s^k
// against all boxes of the node (center-based assignment), the distances to
// the refs (sample-based assignment and the balls of S_+^k), and folds the
// samples into per-box running min / max / count registers. Sharing one load
// of the samples among NG nodes divides the sample traffic of a launch by NG.
// Wavefront shuffles and one integer atomic per value and wavefront finish the
// reduction; floats travel as order-preserving integers, so the results do not
// depend on the order of the atomics, the tile or NG.
#pragma once

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
  int n_chunks, kc;  // boxes per chunk (n_chunks > 1 only with NG = 1)
  int n_groups;      // node groups of NG nodes
  int node_floats;   // LDS floats per node slot
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

// Per node of a workgroup: where its boxes start, how many, whether every box
// has refs, and where each box's refs sit in the node's LDS slot.
struct NodeSlot {
  int b0, cnt, allref;
  int rbeg[64], rcnt[64];
};

// D: attribute count (0 = any, up to 16); KC: boxes per chunk held in
// registers; S: samples per lane per tile; NG: nodes per workgroup; REFS: the
// batch carries refs (without refs none of that code is compiled in); MINW:
// wavefronts per SIMD the register allocation must allow (0 = compiler's
// choice).
template <int D, int KC, int S, int NG, bool REFS, int MINW>
__global__ __launch_bounds__(WG, MINW > 0 ? MINW : 1) void k_tighten(TightenArgs A) {
  constexpr int DM = D ? D : 16;
  const int dd = D ? D : A.d;
  extern __shared__ float sm[];  // per node slot: boxes [k_max][2DM], refs' boxes, refs
  __shared__ NodeSlot s_node[NG];

  const int tid = threadIdx.x, lane = tid & 63;
  const int u = kcd::xcd_unit(blockIdx.x, gridDim.x);
  const int chunk = u % A.n_chunks;
  const int rest = u / A.n_chunks;
  const int grp = rest % A.n_groups, split = rest / A.n_groups;
  const int m0 = grp * NG;

  if (tid < NG) {
    NodeSlot &ns = s_node[tid];
    const int m = m0 + tid;
    int b0 = 0, cnt = 0;
    if (m < A.n_nodes) {
      b0 = kcd::clampi(A.box_off[m], 0, A.n_boxes);
      const int b1 = kcd::clampi(A.box_off[m + 1], b0, A.n_boxes);
      cnt = min(b1 - b0, A.k_max);
    }
    ns.b0 = b0;
    ns.cnt = cnt;
    int all = cnt > 0 && A.ref_off != nullptr;
    int tot = 0;
    for (int k = 0; k < cnt; ++k) {
      int rc = 0;
      if (A.ref_off) {
        const int rb = kcd::clampi(A.ref_off[b0 + k], 0, A.n_refs);
        const int re = kcd::clampi(A.ref_off[b0 + k + 1], rb, A.n_refs);
        rc = min(re - rb, A.max_refs);
      }
      ns.rbeg[k] = tot;  // position in the LDS copy
      ns.rcnt[k] = rc;
      tot += rc;
      if (rc == 0) all = 0;
    }
    ns.allref = all;
  }
  __syncthreads();
  const int box_floats = A.k_max * 2 * DM;
  for (int i = tid; i < NG * A.k_max * DM; i += WG) {
    const int jn = i / (A.k_max * DM);
    const int r = i - jn * A.k_max * DM;
    const int k = r / DM, a = r - k * DM;
    float l = 0.f, h = 0.f;
    if (k < s_node[jn].cnt && a < dd) {
      const int64_t b = s_node[jn].b0 + k;
      l = A.lo[b * dd + a];
      h = A.hi[b * dd + a];
    }
    float *bx = sm + jn * A.node_floats;
    bx[k * 2 * DM + 2 * a] = l;
    bx[k * 2 * DM + 2 * a + 1] = h;
  }
  if (REFS && A.ref_off) {
    // refs of box k of each node are copied densely in box order
    for (int jn = 0; jn < NG; ++jn) {
      float *rf = sm + jn * A.node_floats + 2 * box_floats;
      const int cnt = s_node[jn].cnt, b0 = s_node[jn].b0;
      for (int k = 0; k < cnt; ++k) {
        const int rb = kcd::clampi(A.ref_off[b0 + k], 0, A.n_refs);
        const int rc = s_node[jn].rcnt[k], rp = s_node[jn].rbeg[k];
        for (int i = tid; i < rc * DM; i += WG) {
          const int r = i / DM, a = i - r * DM;
          rf[(rp + r) * DM + a] = a < dd ? A.ref[(int64_t)(rb + r) * dd + a] : 0.f;
        }
      }
    }
  }
  if (REFS) {
    __syncthreads();
    // one lane per (node, box): bounding box of its refs, then the refs
    // holding the smallest or largest value of some attribute moved to the
    // front
    for (int i = tid; i < NG * 64; i += WG) {
      const int jn = i >> 6, k = i & 63;
      if (k >= s_node[jn].cnt) continue;
      float *base = sm + jn * A.node_floats;
      float *R = base + 2 * box_floats + s_node[jn].rbeg[k] * DM;
      float *B = base + box_floats + k * 2 * DM;
      const int rc = s_node[jn].rcnt[k];
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
  float bmin[NG][KC][DM], bmax[NG][KC][DM], amin[NG][KC][DM], amax[NG][KC][DM];
  uint32_t nin[NG][KC], nasg[NG][KC];
  uint64_t far[NG][KC];
  uint32_t nex[NG];
#pragma unroll
  for (int jn = 0; jn < NG; ++jn) {
    nex[jn] = 0;
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      nin[jn][kk] = 0;
      nasg[jn][kk] = 0;
      far[jn][kk] = 0;
#pragma unroll
      for (int a = 0; a < DM; ++a) {
        bmin[jn][kk][a] = INFINITY;
        bmax[jn][kk][a] = -INFINITY;
        amin[jn][kk][a] = INFINITY;
        amax[jn][kk][a] = -INFINITY;
      }
    }
  }
  int cnt_u[NG];
  bool allref[NG];
#pragma unroll
  for (int jn = 0; jn < NG; ++jn) {
    cnt_u[jn] = __builtin_amdgcn_readfirstlane(s_node[jn].cnt);
    allref[jn] = __builtin_amdgcn_readfirstlane(s_node[jn].allref) != 0;
  }
  const bool write_labels = A.labels != nullptr && chunk == 0 && NG == 1;

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

#pragma unroll
    for (int jn = 0; jn < NG; ++jn) {
      if (m0 + jn >= A.n_nodes) break;  // workgroup-uniform
      const float *bx = sm + jn * A.node_floats;
      const float *rbx = bx + box_floats;
      const float *rf = rbx + box_floats;
      const int cnt = cnt_u[jn];
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
          if (k < cnt) {
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
        for (int k = 0; k < cnt; ++k) {
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
          if (k < cnt) {
#pragma unroll
            for (int i = 0; i < S; ++i) {
              bool in = true;
#pragma unroll
              for (int a = 0; a < DM; ++a)
                if (a < dd)
                  in = in && (bx[k * 2 * DM + 2 * a] <= xs[i][a]) &&
                       (xs[i][a] <= bx[k * 2 * DM + 2 * a + 1]);
              inm[i] |= (uint32_t)in << kk;
            }
          }
        }
      }

#pragma unroll
      for (int i = 0; i < S; ++i) {
        const float *xv = xs[i];
        int lab = n_out[i] == cnt ? -2 : (n_out[i] == cnt - 1 ? keep[i] : -1);
        if (base + i >= s_hi) {  // past the end: no contribution
          lab = -3;
          inm[i] = 0;
        }
        // Sample-based assignment (Lemma 2), only for unassigned samples:
        // cluster k is excluded once one of its refs is farther than 4 alpha;
        // the scan stops when two clusters remain possible.
        if (REFS && lab == -1 && allref[jn]) {
          int n_near = 0, rest_k = -1;
          for (int k = 0; k < cnt && n_near < 2; ++k) {
            const int rb = __builtin_amdgcn_readfirstlane(s_node[jn].rbeg[k]);
            const int rc = __builtin_amdgcn_readfirstlane(s_node[jn].rcnt[k]);
            if (all_refs_within(xv, rbx + k * 2 * DM, rf + rb * DM, rc, A.t_sample, dd, DM)) {
              ++n_near;
              rest_k = k;
            }
          }
          if (n_near == 1) lab = rest_k;
        }
        if (write_labels && base + i < s_hi) A.labels[base + i] = (int8_t)lab;
        nex[jn] += (lab == -2);
        label[i] = lab;
      }

      // Running aggregates of the chunk's boxes, box-major.
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) {
        const int k = c0 + kk;
        if (k < cnt) {
          float mid[DM];
#pragma unroll
          for (int a = 0; a < DM; ++a)
            mid[a] = 0.5f * (bx[k * 2 * DM + 2 * a] + bx[k * 2 * DM + 2 * a + 1]);
          const int rb = __builtin_amdgcn_readfirstlane(s_node[jn].rbeg[k]);
          const int rc = __builtin_amdgcn_readfirstlane(s_node[jn].rcnt[k]);
#pragma unroll
          for (int i = 0; i < S; ++i) {
            const float *xv = xs[i];
            if (label[i] == k) {
              ++nasg[jn][kk];
              float dm = 0.f;
#pragma unroll
              for (int a = 0; a < DM; ++a) {
                amin[jn][kk][a] = fminf(amin[jn][kk][a], xv[a]);
                amax[jn][kk][a] = fmaxf(amax[jn][kk][a], xv[a]);
                const float w = xv[a] - mid[a];
                dm = (a == 0) ? w * w : __builtin_fmaf(w, w, dm);
              }
              const uint64_t key = kcd::key_max(dm, (uint32_t)(base + i));
              far[jn][kk] = key > far[jn][kk] ? key : far[jn][kk];
            }
            // S_+^k: inside box k and within the ball of every ref of box k.
            bool in = (inm[i] >> (single ? k : kk)) & 1u;
            if (REFS && in && rc > 0)
              in = all_refs_within(xv, rbx + k * 2 * DM, rf + rb * DM, rc, A.t_ball, dd, DM);
            if (in) {
              ++nin[jn][kk];
#pragma unroll
              for (int a = 0; a < DM; ++a) {
                bmin[jn][kk][a] = fminf(bmin[jn][kk][a], xv[a]);
                bmax[jn][kk][a] = fmaxf(bmax[jn][kk][a], xv[a]);
              }
            }
          }
        }
      }
    }
  }

  // Wavefront reduction, then one atomic per value and wavefront.
#pragma unroll
  for (int jn = 0; jn < NG; ++jn) {
    if (m0 + jn >= A.n_nodes) break;
    const int cnt = cnt_u[jn];
    const int b0 = s_node[jn].b0;
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const int k = c0 + kk;
      const uint32_t ci = kcd::wave_sum_u32(nin[jn][kk]);
      const uint32_t ca = kcd::wave_sum_u32(nasg[jn][kk]);
      const uint64_t fk = kcd::wave_max_u64(far[jn][kk]);
      if (k < cnt) {
        const int64_t b = b0 + k;
        if (lane == 0 && ci) atomicAdd(&A.n_in[b], ci);
        if (lane == 0 && ca) atomicAdd(&A.n_asg[b], ca);
        if (lane == 0 && ca && A.asg_far)
          atomicMax((unsigned long long *)&A.asg_far[b], (unsigned long long)fk);
      }
#pragma unroll
      for (int a = 0; a < DM; ++a) {
        const uint32_t v0 = kcd::wave_min_u32(kcd::ford(bmin[jn][kk][a]));
        const uint32_t v1 = kcd::wave_max_u32(kcd::ford(bmax[jn][kk][a]));
        const uint32_t v2 = kcd::wave_min_u32(kcd::ford(amin[jn][kk][a]));
        const uint32_t v3 = kcd::wave_max_u32(kcd::ford(amax[jn][kk][a]));
        if (k < cnt && a < dd && lane == 0) {
          const int64_t o = (int64_t)(b0 + k) * dd + a;
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
      const uint32_t e = kcd::wave_sum_u32(nex[jn]);
      if (lane == 0 && e) atomicAdd(&A.n_excl[m0 + jn], e);
    }
  }
}

}  // namespace kct

// Compiled variants per attribute count (the autotuner's table). For KC boxes
// per chunk: the default tile (S = 4 samples per lane, 16-byte loads, up to 4
// attributes; 2 beyond), the same held to a register budget of another
// occupancy, half the samples per lane, and -- where the per-node registers
// allow (D * KC <= 20, resp. 8) -- 2 and 4 nodes per workgroup. Chunked
// launches (more boxes than KC) and generic attribute counts use NG = 1.
namespace kct {

constexpr int sdef(int D) { return D > 0 && D <= 4 ? 4 : 2; }
// default wavefronts per SIMD: small shapes hold few aggregates and keep six
// wavefronts resident so that memory latency stays hidden
constexpr int mwdef(int D, int KC) { return D > 0 && D * KC <= 6 ? 6 : 0; }
constexpr int mwalt(int D, int KC) { return mwdef(D, KC) == 4 ? 2 : 4; }

template <int D, int KC, int S, int NG, int MW>
inline bool go(bool refs, const TightenArgs &A, int grid, size_t lds, hipStream_t st) {
  if (refs)
    k_tighten<D, KC, S, NG, true, MW><<<grid, WG, lds, st>>>(A);
  else
    k_tighten<D, KC, S, NG, false, MW><<<grid, WG, lds, st>>>(A);
  return true;
}

template <int D, int KC>
inline bool launch_kc(int S, int NG, int minw, bool refs, const TightenArgs &A, int grid,
                      size_t lds, hipStream_t st) {
  constexpr int SD = sdef(D), MD = mwdef(D, KC), MA = mwalt(D, KC);
  if (S == SD && NG == 1 && minw == MD) return go<D, KC, SD, 1, MD>(refs, A, grid, lds, st);
  if (S == SD && NG == 1 && minw == MA) return go<D, KC, SD, 1, MA>(refs, A, grid, lds, st);
  if (S == SD / 2 && NG == 1 && minw == MD) return go<D, KC, SD / 2, 1, MD>(refs, A, grid, lds, st);
  if constexpr (D > 0 && D * KC <= 20) {
    if (S == SD && NG == 2 && minw == 0) return go<D, KC, SD, 2, 0>(refs, A, grid, lds, st);
    if (S == SD / 2 && NG == 2 && minw == 0) return go<D, KC, SD / 2, 2, 0>(refs, A, grid, lds, st);
  }
  if constexpr (D > 0 && D * KC <= 8) {
    if (S == SD && NG == 4 && minw == 0) return go<D, KC, SD, 4, 0>(refs, A, grid, lds, st);
    if (S == SD / 2 && NG == 4 && minw == 0) return go<D, KC, SD / 2, 4, 0>(refs, A, grid, lds, st);
  }
  return false;
}

}  // namespace kct

// Dispatch of one translation unit: DV_ attributes (0 = generic, up to 16).
#define KC_TIGHTEN_DISPATCH(NAME)                                                        \
  namespace kct {                                                                       \
  bool NAME(int kc, int S, int NG, int minw, bool refs, const TightenArgs &A, int grid, \
            size_t lds, hipStream_t st) {                                               \
    switch (kc) {                                                                       \
      case 1: return launch_kc<DV_, 1>(S, NG, minw, refs, A, grid, lds, st);            \
      case 2: return launch_kc<DV_, 2>(S, NG, minw, refs, A, grid, lds, st);            \
      case 3: return launch_kc<DV_, 3>(S, NG, minw, refs, A, grid, lds, st);            \
      case 4: return launch_kc<DV_, 4>(S, NG, minw, refs, A, grid, lds, st);            \
      case 5: return launch_kc<DV_, 5>(S, NG, minw, refs, A, grid, lds, st);            \
      case 6: return launch_kc<DV_, 6>(S, NG, minw, refs, A, grid, lds, st);            \
      case 8: return launch_kc<DV_, 8>(S, NG, minw, refs, A, grid, lds, st);            \
      default: return false;                                                            \
    }                                                                                   \
  }                                                                                     \
  }
#define KC_TIGHTEN_DISPATCH_GENERIC(NAME)                                                \
  namespace kct {                                                                       \
  bool NAME(int kc, int S, int NG, int minw, bool refs, const TightenArgs &A, int grid, \
            size_t lds, hipStream_t st) {                                               \
    switch (kc) {                                                                       \
      case 1: return launch_kc<0, 1>(S, NG, minw, refs, A, grid, lds, st);              \
      case 2: return launch_kc<0, 2>(S, NG, minw, refs, A, grid, lds, st);              \
      default: return false;                                                            \
    }                                                                                   \
  }                                                                                     \
  }
