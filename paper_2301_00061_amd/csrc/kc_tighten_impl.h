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
  // (node, chunk of LCHUNK samples) pairs the inside-only kernel handled
  // (nullable, [n_nodes][n_lchunks]): there the center-based test provably
  // excludes nothing, so this kernel skips them
  int node_floats;   // LDS floats per node slot
  int64_t span;
  uint32_t *bb_lo, *bb_hi, *asg_min, *asg_max;  // order-preserving encodings
  uint32_t *n_in, *n_asg, *n_excl;
  uint64_t *asg_far;  // per box: max key (dist to midpoint, ~index); may be null
  int8_t *labels;
  const uint8_t *light_map;
  int64_t n_lchunks;
  int lg_kp;  // wide kernel: 2^lg_kp >= k_max lanes per node
};

constexpr int LCHUNK = 4096;  // samples per chunk of the inside-only decisions

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

// Whether every sample of the tile lies within squared distance t of every
// one of the rc refs at r0 (*all) or no sample does (*none), one lane per ref:
// the bounds over the tile are those of sqdist on the tile's extreme
// coordinates.
template <int DM>
__device__ __forceinline__ void refs_class(const float *r0, int rc, float t, const float (&tlo)[DM],
                                           const float (&thi)[DM], int dd, int lane, bool &all,
                                           bool &none) {
  bool f = true, n = false;
  if (lane < rc) {
    const float *r = r0 + lane * DM;
    float rn = 0.f, rx = 0.f;
#pragma unroll
    for (int a = 0; a < DM; ++a) {
      if (a < dd) {
        const float g = fmaxf(fmaxf(r[a] - thi[a], tlo[a] - r[a]), 0.f);
        const float u = fmaxf(thi[a] - r[a], r[a] - tlo[a]);
        rn = (a == 0) ? g * g : __builtin_fmaf(g, g, rn);
        rx = (a == 0) ? u * u : __builtin_fmaf(u, u, rx);
      }
    }
    f = rx <= t;
    n = rn > t;
  }
  all = __ballot(!f) == 0;
  none = __ballot(n) != 0;
}

// One node and one wavefront tile (64 * S consecutive samples, nval of them
// in the split, bounding box [tlo, thi]) settled from the bounding box alone
// where it can be. Lane k classifies box k of the node (whether every or no
// sample of the tile is excluded from the box's cluster by the center-based
// test, or lies inside the box); where the label needs the sample-based test
// and for each box the tile meets, lane r classifies ref r of the box
// (whether every or no sample lies within 4 alpha, resp. alpha, of every
// ref). The bounds over the tile are formed with the per-sample operations in
// the same order, on the tile's extreme coordinates, and float32 rounding is
// monotone, so a bound on the safe side of a threshold gives every sample's
// test the same outcome. When every sample gets the same label, the label's
// aggregates take the tile's bounding box and count (the farthest-from-
// midpoint key runs per sample unless the tile lies nearer the midpoint than
// an earlier tile of the label: fw holds the least distance of such tiles),
// S_+ aggregates of boxes the tile settles likewise, and only the unsettled
// boxes' S_+ tests run per sample. Returns false (nothing updated) when the
// labels differ within the tile; the per-sample path then runs.
template <int D, int KC, int S, bool REFS>
__device__ __forceinline__ bool tile_node(
    const TightenArgs &A, const float (&xs)[S][D ? D : 16], int64_t base, int64_t s_hi, int nval,
    const float (&tlo)[D ? D : 16], const float (&thi)[D ? D : 16], const float *bx,
    const float *rbx, const float *rf, const NodeSlot &ns, int cnt, bool allref, int lane,
    bool write_labels, uint32_t &nex, uint32_t (&nin)[KC], uint32_t (&nasg)[KC],
    uint64_t (&far)[KC], float (&fw)[KC], float (&bmin)[KC][D ? D : 16],
    float (&bmax)[KC][D ? D : 16], float (&amin)[KC][D ? D : 16], float (&amax)[KC][D ? D : 16]) {
  constexpr int DM = D ? D : 16;
  const int dd = D ? D : A.d;
  bool c_out = false, c_keep = false, in_all = false, in_none = false;
  if (lane < cnt) {
    const float *B = bx + lane * 2 * DM;
    float lb = 0.f, ub = 0.f;
    bool ia = true, inn = false;
#pragma unroll
    for (int a = 0; a < DM; ++a) {
      if (a < dd) {
        const float lo = B[2 * a], hi = B[2 * a + 1];
        // least and greatest distance to [lo, hi] over the tile's range
        const float g = fmaxf(fmaxf(lo - thi[a], tlo[a] - hi), 0.f);
        const float u = fmaxf(fmaxf(lo - tlo[a], thi[a] - hi), 0.f);
        lb = (a == 0) ? g * g : __builtin_fmaf(g, g, lb);
        ub = (a == 0) ? u * u : __builtin_fmaf(u, u, ub);
        ia = ia && lo <= tlo[a] && thi[a] <= hi;
        inn = inn || thi[a] < lo || tlo[a] > hi;
      }
    }
    c_out = lb > A.t_center;
    c_keep = !(ub > A.t_center);
    in_all = ia;
    in_none = inn;
  }
  const uint64_t vm = cnt >= 64 ? ~0ull : ((1ull << cnt) - 1ull);
  const uint64_t m_out = __ballot(c_out) & vm, m_keep = __ballot(c_keep) & vm;
  if ((m_out | m_keep) != vm) return false;  // a center-based test differs within the tile
  const int n_out = __popcll(m_out);
  int lab;
  if (n_out == cnt) {
    lab = -2;
  } else if (n_out == cnt - 1) {
    lab = __ffsll((unsigned long long)(vm & ~m_out)) - 1;
  } else {
    lab = -1;
    if (REFS && allref) {
      // sample-based assignment: exactly one cluster with every ref within
      // 4 alpha gives the label (the per-sample scan stops at two)
      int near = 0, first = -1;
      bool mixed = false;
      for (int k = 0; k < cnt && near < 2; ++k) {
        bool all, none;
        refs_class<DM>(rf + __builtin_amdgcn_readfirstlane(ns.rbeg[k]) * DM,
                       __builtin_amdgcn_readfirstlane(ns.rcnt[k]), A.t_sample, tlo, thi, dd, lane,
                       all, none);
        if (all) {
          ++near;
          if (first < 0) first = k;
        } else if (!none) {
          mixed = true;
        }
      }
      if (near < 2) {
        if (mixed) return false;
        if (near == 1) lab = first;
      }
    }
  }
  const uint32_t cnt0 = lane == 0 ? (uint32_t)nval : 0u;  // counts added once per tile
  if (write_labels) {
#pragma unroll
    for (int i = 0; i < S; ++i)
      if (base + i < s_hi) A.labels[base + i] = (int8_t)lab;
  }
  if (lab == -2) nex += cnt0;
  const uint64_t m_ia = __ballot(in_all) & vm, m_in = __ballot(in_none) & vm;
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    if (k >= cnt) continue;
    if (k == lab) {
      nasg[k] += cnt0;
      float mid[DM];
      float lm = 0.f, um = 0.f;
#pragma unroll
      for (int a = 0; a < DM; ++a) {
        amin[k][a] = fminf(amin[k][a], tlo[a]);
        amax[k][a] = fmaxf(amax[k][a], thi[a]);
        mid[a] = 0.5f * (bx[k * 2 * DM + 2 * a] + bx[k * 2 * DM + 2 * a + 1]);
        if (a < dd) {
          // least and greatest distance to the midpoint over the tile
          const float g = fmaxf(fmaxf(mid[a] - thi[a], tlo[a] - mid[a]), 0.f);
          const float u = fmaxf(thi[a] - mid[a], mid[a] - tlo[a]);
          lm = (a == 0) ? g * g : __builtin_fmaf(g, g, lm);
          um = (a == 0) ? u * u : __builtin_fmaf(u, u, um);
        }
      }
      // an earlier tile of this label holds a sample farther from the
      // midpoint than any sample of this one: the key cannot change
      if (!(um < fw[k])) {
#pragma unroll
        for (int i = 0; i < S; ++i) {
          if (base + i >= s_hi) continue;
          float dm = 0.f;
#pragma unroll
          for (int a = 0; a < DM; ++a) {
            if (a < dd) {
              const float w = xs[i][a] - mid[a];
              dm = (a == 0) ? w * w : __builtin_fmaf(w, w, dm);
            }
          }
          const uint64_t key = kcd::key_max(dm, (uint32_t)(base + i));
          far[k] = key > far[k] ? key : far[k];
        }
      }
      fw[k] = fmaxf(fw[k], lm);
    }
    // S_+^k: inside box k and within the ball of every ref of box k
    const uint64_t bit = 1ull << k;
    if (m_in & bit) continue;
    const int rb = __builtin_amdgcn_readfirstlane(ns.rbeg[k]);
    const int rc = REFS ? __builtin_amdgcn_readfirstlane(ns.rcnt[k]) : 0;
    bool ball_all = true, ball_none = false;
    if (REFS && rc > 0) refs_class<DM>(rf + rb * DM, rc, A.t_ball, tlo, thi, dd, lane, ball_all, ball_none);
    if (ball_none) continue;
    if ((m_ia & bit) && ball_all) {
      nin[k] += cnt0;
#pragma unroll
      for (int a = 0; a < DM; ++a) {
        bmin[k][a] = fminf(bmin[k][a], tlo[a]);
        bmax[k][a] = fmaxf(bmax[k][a], thi[a]);
      }
      continue;
    }
#pragma unroll
    for (int i = 0; i < S; ++i) {
      bool in = base + i < s_hi;
#pragma unroll
      for (int a = 0; a < DM; ++a)
        if (a < dd)
          in = in && (bx[k * 2 * DM + 2 * a] <= xs[i][a]) && (xs[i][a] <= bx[k * 2 * DM + 2 * a + 1]);
      if (REFS && in && rc > 0)
        in = all_refs_within(xs[i], rbx + k * 2 * DM, rf + rb * DM, rc, A.t_ball, dd, DM);
      if (in) {
        ++nin[k];
#pragma unroll
        for (int a = 0; a < DM; ++a) {
          bmin[k][a] = fminf(bmin[k][a], xs[i][a]);
          bmax[k][a] = fmaxf(bmax[k][a], xs[i][a]);
        }
      }
    }
  }
  return true;
}

// Stages the boxes of nodes m0 .. m0 + NG - 1 in LDS (node slot jn at
// sm + jn * node_floats: boxes [k_max][2DM], their refs' bounding boxes
// [k_max][2DM], then the refs), with each box's refs holding the smallest or
// largest value of some attribute moved to the front. Ends with a barrier.
template <int DM, int NG, bool REFS>
__device__ __forceinline__ void stage_nodes(const TightenArgs &A, int m0, NodeSlot *s_node,
                                            float *sm, int dd, int tid) {
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
}

// D: attribute count (0 = any, up to 16); KC: boxes per chunk held in
// registers; S: samples per lane per tile; NG: nodes per workgroup; REFS: the
// batch carries refs (without refs none of that code is compiled in); MINW:
// wavefronts per SIMD the register allocation must allow (0 = compiler's
// choice); TSKIP: wavefront tiles that the bounding box of their samples
// settles skip the per-sample tests (single-chunk launches only).
template <int D, int KC, int S, int NG, bool REFS, int MINW, bool TSKIP>
__global__ __launch_bounds__(WG, MINW > 0 ? MINW : 1) void k_tighten(TightenArgs A) {
  constexpr int DM = D ? D : 16;
  constexpr int SC = S < 4 ? S : 4;  // samples per chunk of the per-sample path
  const int dd = D ? D : A.d;
  extern __shared__ float sm[];  // per node slot: boxes [k_max][2DM], refs' boxes, refs
  __shared__ NodeSlot s_node[NG];

  const int tid = threadIdx.x, lane = tid & 63;
  const int u = kcd::xcd_unit(blockIdx.x, gridDim.x);
  const int chunk = u % A.n_chunks;
  const int rest = u / A.n_chunks;
  const int grp = rest % A.n_groups, split = rest / A.n_groups;
  const int m0 = grp * NG;

  stage_nodes<DM, NG, REFS>(A, m0, s_node, sm, dd, tid);
  const int box_floats = A.k_max * 2 * DM;

  const int c0 = chunk * A.kc;
  const bool single = A.n_chunks == 1;
  float bmin[NG][KC][DM], bmax[NG][KC][DM], amin[NG][KC][DM], amax[NG][KC][DM];
  uint32_t nin[NG][KC], nasg[NG][KC];
  uint64_t far[NG][KC];
  float fw[NG][KC];  // tile decisions: at most the farthest folded distance to the midpoint
  uint32_t nex[NG];
#pragma unroll
  for (int jn = 0; jn < NG; ++jn) {
    nex[jn] = 0;
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      nin[jn][kk] = 0;
      nasg[jn][kk] = 0;
      far[jn][kk] = 0;
      fw[jn][kk] = -1.f;
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
  static_assert(LCHUNK % (64 * S) == 0, "a wavefront's tile lies in one chunk");

  const int64_t s_lo = (int64_t)split * A.span;
  const int64_t s_hi = min(A.n, s_lo + A.span);
  const int wave = tid >> 6;
  // With tile decisions every lane runs the same number of tiles (the last
  // tile of a split may hold samples past its end, which take no part), so
  // that the wavefront decisions see whole wavefronts; without, a lane stops
  // after its last sample.
  const int64_t lane_off = (int64_t)tid * S;
  for (int64_t base = s_lo + lane_off; (TSKIP ? base - lane_off : base) < s_hi;
       base += (int64_t)WG * S) {
    const int64_t tb = base - lane_off;
    float xs[S][DM];
    const bool full = base + S <= s_hi;
#pragma unroll
    for (int a = 0; a < DM; ++a) {
      if (a < dd) {
        const float *p = A.x + (int64_t)a * A.ld + base;
        if (full && S % 4 == 0) {
#pragma unroll
          for (int q = 0; q < S / 4; ++q) {
            const float4 v = reinterpret_cast<const float4 *>(p)[q];
            xs[(4 * q) % S][a] = v.x;
            xs[(4 * q + 1) % S][a] = v.y;
            xs[(4 * q + 2) % S][a] = v.z;
            xs[(4 * q + 3) % S][a] = v.w;
          }
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
    // Wavefront tile: the 64 * S consecutive samples of this wavefront, their
    // count and bounding box (uniform across the wavefront).
    int nval = 0;
    float tlo[DM], thi[DM];
    if constexpr (TSKIP) {
      const int64_t wb = tb + (int64_t)wave * 64 * S;
      const int64_t left = s_hi - wb;
      nval = left <= 0 ? 0 : (left >= 64 * S ? 64 * S : (int)left);
#pragma unroll
      for (int a = 0; a < DM; ++a) {
        float l = INFINITY, h = -INFINITY;
        if (a < dd) {
#pragma unroll
          for (int i = 0; i < S; ++i)
            if (base + i < s_hi) {
              l = fminf(l, xs[i][a]);
              h = fmaxf(h, xs[i][a]);
            }
        }
        tlo[a] = __int_as_float(__builtin_amdgcn_readfirstlane(
            __float_as_int(kcd::fdec(kcd::wave_min_u32(kcd::ford(l))))));
        thi[a] = __int_as_float(__builtin_amdgcn_readfirstlane(
            __float_as_int(kcd::fdec(kcd::wave_max_u32(kcd::ford(h))))));
      }
    }

#pragma unroll
    for (int jn = 0; jn < NG; ++jn) {
      if (m0 + jn >= A.n_nodes) break;  // workgroup-uniform
      if (A.light_map && tb + (int64_t)wave * 64 * S < s_hi &&
          A.light_map[(int64_t)(m0 + jn) * A.n_lchunks + (tb + (int64_t)wave * 64 * S) / LCHUNK])
        continue;  // the inside-only kernel took this node's chunk
      bool done = false;
      if constexpr (TSKIP) {
        if (nval == 0) {
          done = true;  // no sample of this wavefront lies in the split
        } else {
          const float *bx = sm + jn * A.node_floats;
          const float *rbx = bx + box_floats;
          const float *rf = rbx + box_floats;
          const int cnt = cnt_u[jn];
          done = tile_node<D, KC, S, REFS>(A, xs, base, s_hi, nval, tlo, thi, bx, rbx, rf,
                                           s_node[jn], cnt, allref[jn], lane, write_labels,
                                           nex[jn], nin[jn], nasg[jn], far[jn], fw[jn], bmin[jn],
                                           bmax[jn], amin[jn], amax[jn]);
        }
      }
      if (!done) {
        // per-sample path, in chunks of SC samples of the lane
#pragma unroll
        for (int i0 = 0; i0 < S; i0 += SC) {
          const float *bx = sm + jn * A.node_floats;
          const float *rbx = bx + box_floats;
          const float *rf = rbx + box_floats;
          const int cnt = cnt_u[jn];
          // Center-based assignment (Lemma 1), box-major: each box's bounds are
          // read from LDS once for the lane's SC samples. In the single-chunk case
          // the same distances record which boxes hold each sample.
          int n_out[SC], keep[SC], label[SC];
          uint32_t inm[SC];
#pragma unroll
          for (int i = 0; i < SC; ++i) {
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
                for (int i = 0; i < SC; ++i) {
                  float acc = 0.f;
                  bool in = true;
#pragma unroll
                  for (int a = 0; a < DM; ++a) {
                    if (a < dd) {
                      const float c = kcd::med3(lo[a], xs[i0 + i][a], hi[a]);
                      in = in && (c == xs[i0 + i][a]);
                      const float t = xs[i0 + i][a] - c;
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
              for (int i = 0; i < SC; ++i) {
                float acc = 0.f;
#pragma unroll
                for (int a = 0; a < DM; ++a) {
                  if (a < dd) {
                    const float t = xs[i0 + i][a] - kcd::med3(lo[a], xs[i0 + i][a], hi[a]);
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
                for (int i = 0; i < SC; ++i) {
                  bool in = true;
#pragma unroll
                  for (int a = 0; a < DM; ++a)
                    if (a < dd)
                      in = in && (bx[k * 2 * DM + 2 * a] <= xs[i0 + i][a]) &&
                           (xs[i0 + i][a] <= bx[k * 2 * DM + 2 * a + 1]);
                  inm[i] |= (uint32_t)in << kk;
                }
              }
            }
          }

#pragma unroll
          for (int i = 0; i < SC; ++i) {
            const float *xv = xs[i0 + i];
            int lab = n_out[i] == cnt ? -2 : (n_out[i] == cnt - 1 ? keep[i] : -1);
            if (base + i0 + i >= s_hi) {  // past the end: no contribution
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
            if (write_labels && base + i0 + i < s_hi) A.labels[base + i0 + i] = (int8_t)lab;
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
              for (int i = 0; i < SC; ++i) {
                const float *xv = xs[i0 + i];
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
                  const uint64_t key = kcd::key_max(dm, (uint32_t)(base + i0 + i));
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

// Wide variants (S, NG): usable when NG << lg_kp <= 64.
#define KCT_WIDE_VARIANTS(X) X(8, 4) X(8, 8) X(8, 16) X(16, 4) X(16, 8) X(16, 16)
#include "kc_tighten_wide.h"

// Compiled variants per attribute count (the autotuner's table). For KC boxes
// per chunk: the default tile (S = 4 samples per lane, 16-byte loads, up to 4
// attributes; 2 beyond), the same held to a register budget of another
// occupancy, half the samples per lane, 2 nodes per workgroup where the
// per-node registers allow (D * KC <= 20); and with wavefront tiles settled
// from their bounding box: 1, 2 and 4 times the default samples per lane, and
// 2 nodes per workgroup with 1 or 2 times. Chunked launches (more boxes than
// KC) and generic attribute counts use NG = 1 without tile decisions.
namespace kct {

constexpr int sdef(int D) { return D > 0 && D <= 4 ? 4 : 2; }
// default wavefronts per SIMD: small shapes hold few aggregates and keep six
// wavefronts resident so that memory latency stays hidden
constexpr int mwdef(int D, int KC) { return D > 0 && D * KC <= 6 ? 6 : 0; }
constexpr int mwalt(int D, int KC) { return mwdef(D, KC) == 4 ? 2 : 4; }

template <int D, int KC, int S, int NG, int MW, bool SK>
inline bool go(bool refs, const TightenArgs &A, int grid, size_t lds, hipStream_t st) {
  if (refs)
    k_tighten<D, KC, S, NG, true, MW, SK><<<grid, WG, lds, st>>>(A);
  else
    k_tighten<D, KC, S, NG, false, MW, SK><<<grid, WG, lds, st>>>(A);
  return true;
}

template <int D, int KC>
inline bool launch_kc(int S, int NG, int minw, int skip, bool refs, const TightenArgs &A, int grid,
                      size_t lds, hipStream_t st) {
  constexpr int SD = sdef(D), MD = mwdef(D, KC), MA = mwalt(D, KC);
  if (!skip) {
    if (S == SD && NG == 1 && minw == MD) return go<D, KC, SD, 1, MD, false>(refs, A, grid, lds, st);
    if (S == SD && NG == 1 && minw == MA) return go<D, KC, SD, 1, MA, false>(refs, A, grid, lds, st);
    if (S == SD / 2 && NG == 1 && minw == MD)
      return go<D, KC, SD / 2, 1, MD, false>(refs, A, grid, lds, st);
    if constexpr (D > 0 && D * KC <= 20) {
      if (S == SD && NG == 2 && minw == 0) return go<D, KC, SD, 2, 0, false>(refs, A, grid, lds, st);
    }
  } else if constexpr (D > 0) {
    // wavefront tiles (64 S samples) settled from their bounding box
    if (NG == 1 && minw == 0) {
      if (S == SD) return go<D, KC, SD, 1, 0, true>(refs, A, grid, lds, st);
      if (S == 2 * SD) return go<D, KC, 2 * SD, 1, 0, true>(refs, A, grid, lds, st);
      if (S == 4 * SD) return go<D, KC, 4 * SD, 1, 0, true>(refs, A, grid, lds, st);
    }
    if constexpr (D * KC <= 20) {
      if (NG == 2 && minw == 0) {
        if (S == SD) return go<D, KC, SD, 2, 0, true>(refs, A, grid, lds, st);
        if (S == 2 * SD) return go<D, KC, 2 * SD, 2, 0, true>(refs, A, grid, lds, st);
      }
    }
  }
  return false;
}

}  // namespace kct

// Dispatch of one translation unit: DV_ attributes (0 = generic, up to 16).
#define KC_TIGHTEN_DISPATCH(NAME)                                                        \
  namespace kct {                                                                       \
  bool NAME(int kc, int S, int NG, int minw, int skip, bool refs, const TightenArgs &A,   \
            int grid, size_t lds, hipStream_t st) {                                     \
    if (skip == 2) return launch_wide<DV_>(S, NG, minw >= 1000, refs, A, grid, lds, st);\
    switch (kc) {                                                                       \
      case 1: return launch_kc<DV_, 1>(S, NG, minw, skip, refs, A, grid, lds, st);      \
      case 2: return launch_kc<DV_, 2>(S, NG, minw, skip, refs, A, grid, lds, st);      \
      case 3: return launch_kc<DV_, 3>(S, NG, minw, skip, refs, A, grid, lds, st);      \
      case 4: return launch_kc<DV_, 4>(S, NG, minw, skip, refs, A, grid, lds, st);      \
      case 5: return launch_kc<DV_, 5>(S, NG, minw, skip, refs, A, grid, lds, st);      \
      case 6: return launch_kc<DV_, 6>(S, NG, minw, skip, refs, A, grid, lds, st);      \
      case 8: return launch_kc<DV_, 8>(S, NG, minw, skip, refs, A, grid, lds, st);      \
      default: return false;                                                            \
    }                                                                                   \
  }                                                                                     \
  }
#define KC_TIGHTEN_DISPATCH_GENERIC(NAME)                                                \
  namespace kct {                                                                       \
  bool NAME(int kc, int S, int NG, int minw, int skip, bool refs, const TightenArgs &A,   \
            int grid, size_t lds, hipStream_t st) {                                     \
    switch (kc) {                                                                       \
      case 1: return launch_kc<0, 1>(S, NG, minw, skip, refs, A, grid, lds, st);        \
      case 2: return launch_kc<0, 2>(S, NG, minw, skip, refs, A, grid, lds, st);        \
      default: return false;                                                            \
    }                                                                                   \
  }                                                                                     \
  }
