// kc_bound_impl.h -- the streaming bound kernels (templates; instantiated per
// attribute count in kc_bound_d*.hip).
//
// k_bound evaluates, for a batch of nodes (each a set of center boxes),
//     beta(M) = max_s min_k sum_a (x_{s,a} - mid{lo_a^k, x_{s,a}, hi_a^k})^2
// (Section 3.1, eqs (8)-(11)) with its argmax, optionally the Section 3.2
// upper-bound candidates (per box, the sample inside it closest to its
// midpoint), and -- with POINT, where every box is a single point -- the
// objective of eq (12).
//
// Work decomposition: a workgroup owns NG consecutive nodes (their boxes are
// staged in LDS, their running maxima live in registers) and one contiguous
// split of the samples, which its 256 lanes stream in tiles of 256*S samples
// with 16-byte loads of each structure-of-arrays row. Per lane the samples are
// visited in increasing index order, so a strict '>' keeps the lowest index
// among equal maxima. At the end every wavefront reduces packed (value,index)
// keys with cross-lane shuffles, the workgroup combines its four wavefronts in
// LDS and writes one partial key per node; k_bound_finalize reduces the
// partials of all splits. No float atomics: results are bit-reproducible.
#pragma once

#include "kc_device.h"
#include "kc_internal.h"

namespace kcb {

constexpr int WG = 256;
constexpr int NWAVE = WG / kcd::WAVE;

struct BoundArgs {
  const float *x;
  int64_t n, ld;
  int d;
  int n_nodes, n_boxes, k_max;
  const int32_t *box_off;  // null in POINT mode: node m owns boxes m*k_max ..
  const float *lo, *hi;    // hi unused in POINT mode
  int n_groups;
  int64_t span;            // samples per split (multiple of WG*S)
  int lg_kp;               // tile decisions: 2^lg_kp >= k_max lanes per node
  // POINT screening (dead non-null): a set whose value exceeds `cut` may
  // stop early; dead[m] != 0 once some wavefront has folded a value above
  // the cut for set m (read and written by all workgroups).
  float cut;
  uint32_t *dead;
  // POINT with tile decisions (nullable): a lower bound of each set's exact
  // objective; lowered by the float32 margin (frel, fabs) it is a value the
  // set's float32 maximum reaches, so tiles strictly below it are skipped
  const double *floor;
  double frel, fabs_;
  // POINT screening (nullable): per set one sample (coordinates [n_nodes][d]
  // and its index in x); a set whose value at it exceeds the cut is settled
  // at that value before any tile
  const float *wit_x;
  const int64_t *wit_id;
  // tile decisions: per node the largest W and per box the least cw any
  // wavefront has published (order-preserving encodings; null = no sharing)
  uint32_t *gW, *gC;
  uint64_t *part_key;      // [splits][n_nodes]
  uint64_t *part_cand;     // [splits][n_boxes] (candidate variants)
};

// The variants with wavefront tile decisions are k_bound_wide (kc_bound_wide.h).
template <int D, int S, int NG, int KC, bool POINT>
__global__ __launch_bounds__(WG) void k_bound(BoundArgs A) {
  constexpr int DM = D ? D : 16;
  constexpr int KCA = KC > 0 ? KC : 1;
  const int dd = D ? D : A.d;
  extern __shared__ float smem[];  // [NG][k_max][DM] interleaved (lo, hi)
  __shared__ int s_beg[NG], s_cnt[NG];
  __shared__ uint64_t s_red[NWAVE][NG];
  __shared__ uint64_t s_cred[NWAVE][KC > 0 ? NG * KC : 1];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int u = kcd::xcd_unit(blockIdx.x, gridDim.x);
  const int g = u % A.n_groups, split = u / A.n_groups;
  const int m0 = g * NG;

  if (tid < NG) {
    const int m = m0 + tid;
    int b0 = 0, c = 0;
    if (m < A.n_nodes) {
      if (POINT) {
        b0 = m * A.k_max;
        c = A.k_max;
      } else {
        b0 = kcd::clampi(A.box_off[m], 0, A.n_boxes);
        const int b1 = kcd::clampi(A.box_off[m + 1], b0, A.n_boxes);
        c = min(b1 - b0, A.k_max);
      }
    }
    s_beg[tid] = b0;
    s_cnt[tid] = c;
  }
  __syncthreads();
  const int per_node = A.k_max * 2 * DM;
  for (int i = tid; i < NG * A.k_max * DM; i += WG) {
    const int jn = i / (A.k_max * DM);
    const int r = i - jn * A.k_max * DM;
    const int k = r / DM, a = r - k * DM;
    float l = 0.0f, h = 0.0f;
    if (k < s_cnt[jn] && a < dd) {
      const int64_t b = s_beg[jn] + k;
      l = A.lo[b * dd + a];
      h = POINT ? l : A.hi[b * dd + a];
    }
    smem[jn * per_node + k * 2 * DM + 2 * a] = l;
    smem[jn * per_node + k * 2 * DM + 2 * a + 1] = h;
  }
  __syncthreads();

  float rmax[NG];
  uint32_t ridx[NG];
  float cmin[NG][KCA];
  uint32_t cidx[NG][KCA];
#pragma unroll
  for (int j = 0; j < NG; ++j) {
    rmax[j] = -1.0f;
    ridx[j] = 0;
#pragma unroll
    for (int k = 0; k < KCA; ++k) {
      cmin[j][k] = INFINITY;
      cidx[j][k] = 0xffffffffu;
    }
  }

  uint64_t deadm = 0;  // screening: bit jn, set jn already exceeds the cut
  int tick = 0;

  const int64_t s_lo = (int64_t)split * A.span;
  const int64_t s_hi = min(A.n, s_lo + A.span);
  const int64_t lane_off = (int64_t)tid * S;
  for (int64_t base = s_lo + lane_off; base < s_hi; base += (int64_t)WG * S) {
    float xv[DM][S];
    const bool full = base + S <= s_hi;
#pragma unroll
    for (int a = 0; a < DM; ++a) {
      if (a < dd) {
        const float *p = A.x + (int64_t)a * A.ld + base;
        if (full) {
          if constexpr (S % 4 == 0) {
#pragma unroll
            for (int q = 0; q < S / 4; ++q) {
              const float4 v = reinterpret_cast<const float4 *>(p)[q];
              xv[a][4 * q] = v.x;
              xv[a][4 * q + 1] = v.y;
              xv[a][4 * q + 2] = v.z;
              xv[a][4 * q + 3] = v.w;
            }
          } else if constexpr (S == 2) {
            const float2 v = *reinterpret_cast<const float2 *>(p);
            xv[a][0] = v.x;
            xv[a][1] = v.y;
          } else {
#pragma unroll
            for (int i = 0; i < S; ++i) xv[a][i] = p[i];
          }
        } else {
#pragma unroll
          for (int i = 0; i < S; ++i) xv[a][i] = (base + i < s_hi) ? p[i] : 0.0f;
        }
      } else {
#pragma unroll
        for (int i = 0; i < S; ++i) xv[a][i] = 0.0f;
      }
    }

    const bool refresh = (tick++ & 15) == 0;
    if constexpr (POINT) {
      // every 16th tile: sets that other workgroups found above the cut
      if (A.dead && refresh) {
        uint32_t f = 0;
        if (lane < NG && m0 + lane < A.n_nodes)
          f = __hip_atomic_load(A.dead + m0 + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        deadm |= __ballot(f != 0u);
      }
    }

#pragma unroll
    for (int jn = 0; jn < NG; ++jn) {
      if (m0 + jn >= A.n_nodes) break;
      const float *bx = smem + jn * per_node;
      const int cnt = s_cnt[jn];
      if (POINT && ((deadm >> jn) & 1ull)) continue;
      float best[S];
#pragma unroll
      for (int i = 0; i < S; ++i) best[i] = INFINITY;

      if constexpr (KC == 0) {
        for (int k = 0; k < cnt; ++k) {
          float l[DM], h[DM];
#pragma unroll
          for (int a = 0; a < DM; ++a) {
            l[a] = bx[k * 2 * DM + 2 * a];
            h[a] = bx[k * 2 * DM + 2 * a + 1];
          }
#pragma unroll
          for (int i = 0; i < S; ++i) {
            float acc = 0.0f;
#pragma unroll
            for (int a = 0; a < DM; ++a) {
              if (a < dd) {
                const float c = POINT ? l[a] : kcd::med3(l[a], xv[a][i], h[a]);
                const float t = xv[a][i] - c;
                acc = (a == 0) ? t * t : __builtin_fmaf(t, t, acc);
              }
            }
            best[i] = fminf(best[i], acc);
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < KC; ++k) {
          if (k < cnt) {
            float l[DM], h[DM];
#pragma unroll
            for (int a = 0; a < DM; ++a) {
              l[a] = bx[k * 2 * DM + 2 * a];
              h[a] = bx[k * 2 * DM + 2 * a + 1];
            }
            bool in[S];
#pragma unroll
            for (int i = 0; i < S; ++i) {
              float acc = 0.0f;
              in[i] = base + i < s_hi;
#pragma unroll
              for (int a = 0; a < DM; ++a) {
                if (a < dd) {
                  const float c = kcd::med3(l[a], xv[a][i], h[a]);
                  in[i] = in[i] && (c == xv[a][i]);
                  const float t = xv[a][i] - c;
                  acc = (a == 0) ? t * t : __builtin_fmaf(t, t, acc);
                }
              }
              best[i] = fminf(best[i], acc);
            }
            // distance to the midpoint only when some lane holds a sample
            // inside the box (a wavefront-uniform branch)
            bool any = false;
#pragma unroll
            for (int i = 0; i < S; ++i) any = any || in[i];
            if (__ballot(any)) {
#pragma unroll
              for (int i = 0; i < S; ++i) {
                float dm = 0.0f;
#pragma unroll
                for (int a = 0; a < DM; ++a) {
                  if (a < dd) {
                    const float w = xv[a][i] - 0.5f * (l[a] + h[a]);
                    dm = (a == 0) ? w * w : __builtin_fmaf(w, w, dm);
                  }
                }
                if (in[i] && dm < cmin[jn][k]) {
                  cmin[jn][k] = dm;
                  cidx[jn][k] = (uint32_t)(base + i);
                }
              }
            }
          }
        }
      }
#pragma unroll
      for (int i = 0; i < S; ++i) {
        if (base + i < s_hi && best[i] > rmax[jn]) {
          rmax[jn] = best[i];
          ridx[jn] = (uint32_t)(base + i);
        }
      }
      if constexpr (POINT) {
        // screening: a value above the cut is folded; the set stops here and,
        // through dead[], in the other workgroups
        if (A.dead && __ballot(rmax[jn] > A.cut)) {
          deadm |= 1ull << jn;
          if (lane == 0)
            __hip_atomic_store(A.dead + m0 + jn, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
  }

#pragma unroll
  for (int jn = 0; jn < NG; ++jn) {
    const uint64_t key = kcd::wave_max_u64(kcd::key_max(rmax[jn], ridx[jn]));
    if (lane == 0) s_red[wave][jn] = key;
    if constexpr (KC > 0) {
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        const uint64_t ck = kcd::wave_min_u64(kcd::key_min(cmin[jn][k], cidx[jn][k]));
        if (lane == 0) s_cred[wave][jn * KC + k] = ck;
      }
    }
  }
  __syncthreads();
  if (tid < NG && m0 + tid < A.n_nodes) {
    uint64_t key = s_red[0][tid];
#pragma unroll
    for (int w = 1; w < NWAVE; ++w) key = s_red[w][tid] > key ? s_red[w][tid] : key;
    A.part_key[(int64_t)split * A.n_nodes + m0 + tid] = key;
  }
  if constexpr (KC > 0) {
    for (int i = tid; i < NG * KC; i += WG) {
      const int jn = i / KC, k = i - jn * KC;
      if (m0 + jn < A.n_nodes && k < s_cnt[jn]) {
        uint64_t ck = s_cred[0][i];
#pragma unroll
        for (int w = 1; w < NWAVE; ++w) ck = s_cred[w][i] < ck ? s_cred[w][i] : ck;
        A.part_cand[(int64_t)split * A.n_boxes + s_beg[jn] + k] = ck;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Float64 objective (certificate): obj[c] = max_s min_j ||x_s - c_j||^2 with
// each squared distance formed as ((x0-c0)^2 + (x1-c1)^2) + ... in attribute
// order, every operation correctly rounded and none fused.
struct Obj64Args {
  const float *x;
  int64_t n, ld;
  int d, n_sets, k;
  const float *centers;  // [n_sets][k][d]
  int64_t span;
  double *part_val;      // [splits][n_sets]
  uint32_t *part_idx;    // [splits][n_sets]
};

template <int D>
__global__ __launch_bounds__(WG) void k_obj64(Obj64Args A) {
#pragma clang fp contract(off)
  constexpr int DM = D ? D : 16;
  const int dd = D ? D : A.d;
  extern __shared__ double cs[];  // [k][DM] of set c
  __shared__ double s_v[NWAVE];
  __shared__ uint32_t s_i[NWAVE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = blockIdx.y, split = blockIdx.x;
  for (int i = tid; i < A.k * DM; i += WG) {
    const int j = i / DM, a = i - j * DM;
    cs[i] = a < dd ? (double)A.centers[((int64_t)c * A.k + j) * dd + a] : 0.0;
  }
  __syncthreads();
  double best = -1.0;
  uint32_t bidx = 0xffffffffu;
  const int64_t s_lo = (int64_t)split * A.span;
  const int64_t s_hi = min(A.n, s_lo + A.span);
  for (int64_t s = s_lo + tid; s < s_hi; s += WG) {
    double xv[DM];
#pragma unroll
    for (int a = 0; a < DM; ++a) xv[a] = a < dd ? (double)A.x[(int64_t)a * A.ld + s] : 0.0;
    double q = INFINITY;
    for (int j = 0; j < A.k; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int a = 0; a < DM; ++a) {
        if (a < dd) {
          const double t = xv[a] - cs[j * DM + a];
          const double sq = t * t;
          acc = acc + sq;
        }
      }
      q = q < acc ? q : acc;
    }
    if (q > best) {
      best = q;
      bidx = (uint32_t)s;
    }
  }
  // wave reduction: larger value wins, then lower index
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    const double ov = __shfl_xor(best, m);
    const uint32_t oi = __shfl_xor(bidx, m);
    if (ov > best || (ov == best && oi < bidx)) {
      best = ov;
      bidx = oi;
    }
  }
  if (lane == 0) {
    s_v[wave] = best;
    s_i[wave] = bidx;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < NWAVE; ++w)
      if (s_v[w] > best || (s_v[w] == best && s_i[w] < bidx)) {
        best = s_v[w];
        bidx = s_i[w];
      }
    A.part_val[(int64_t)split * A.n_sets + c] = best;
    A.part_idx[(int64_t)split * A.n_sets + c] = bidx;
  }
}

}  // namespace kcb

#include "kc_bound_wide.h"

// Launch variants: (S, NG) for the lower bound and the float32 objective,
// (S, NG, KC) for the lower bound with candidates (KC >= boxes per node).
#define KCB_LB_VARIANTS(X) X(8, 1) X(4, 1) X(2, 1) X(4, 2) X(4, 4) X(2, 4) X(4, 8) X(2, 8) X(2, 16) X(1, 16)
#define KCB_PT_VARIANTS(X) X(4, 1) X(2, 4) X(2, 8)
#define KCB_CAND_VARIANTS(X) \
  X(2, 8, 4) X(2, 4, 4) X(2, 1, 4) X(4, 4, 4) X(4, 2, 4) X(2, 4, 8) X(2, 2, 8) X(2, 1, 8)       \
  X(4, 2, 8) X(1, 4, 8) X(1, 2, 16) X(1, 1, 16) X(1, 1, 64)

#define KCB_LB_CASE(SV, NGV) \
  if (S == SV && NG == NGV) { k_bound<DV_, SV, NGV, 0, false><<<g, b, lds, st>>>(A); return KC_OK; }
#define KCB_PT_CASE(SV, NGV) \
  if (S == SV && NG == NGV) { k_bound<DV_, SV, NGV, 0, true><<<g, b, lds, st>>>(A); return KC_OK; }
#define KCB_CAND_CASE(SV, NGV, KCV) \
  if (S == SV && NG == NGV && KC == KCV) { k_bound<DV_, SV, NGV, KCV, false><<<g, b, lds, st>>>(A); return KC_OK; }

// Variants with tile decisions (k_bound_wide; attribute counts 1..8; usable
// when NG << lg_kp <= 64).
#define KCB_LB_TS_VARIANTS(X) X(8, 16) X(4, 16) X(8, 8) X(4, 8) X(4, 4) X(8, 1)
#define KCB_PT_TS_VARIANTS(X) X(16, 16) X(8, 16) X(4, 16) X(32, 8) X(16, 8) X(8, 8) X(4, 8) X(4, 4) X(8, 1)
#define KCB_CAND_TS_VARIANTS(X) \
  X(32, 16, 4) X(16, 16, 4) X(8, 16, 4) X(4, 16, 4) X(2, 16, 4) X(16, 8, 4) X(8, 8, 4) X(4, 8, 4) X(8, 8, 8) \
  X(4, 8, 8) X(2, 8, 8) \
  X(4, 4, 8) X(4, 4, 16) X(2, 4, 16) X(4, 1, 64)
#define KCB_LB_TS_CASE(SV, NGV) \
  if (S == SV && NG == NGV) { k_bound_wide<DV, SV, NGV, 0, false><<<g, b, lds, st>>>(A); return KC_OK; }
#define KCB_PT_TS_CASE(SV, NGV) \
  if (S == SV && NG == NGV) { k_bound_wide<DV, SV, NGV, 0, true><<<g, b, lds, st>>>(A); return KC_OK; }
#define KCB_CAND_TS_CASE(SV, NGV, KCV) \
  if (S == SV && NG == NGV && KC == KCV) { k_bound_wide<DV, SV, NGV, KCV, false><<<g, b, lds, st>>>(A); return KC_OK; }

namespace kcb {
template <int DV>
inline kc_status launch_ts(int S, int NG, int KC, bool point, const BoundArgs &A, int grid,
                           size_t lds, hipStream_t st) {
  if constexpr (DV > 0) {
    dim3 g(grid), b(WG);
    if (point) {
      KCB_PT_TS_VARIANTS(KCB_PT_TS_CASE)
      return KC_EUNSUPPORTED;
    }
    if (KC > 0) {
      KCB_CAND_TS_VARIANTS(KCB_CAND_TS_CASE)
      return KC_EUNSUPPORTED;
    }
    KCB_LB_TS_VARIANTS(KCB_LB_TS_CASE)
  }
  return KC_EUNSUPPORTED;
}
}  // namespace kcb

// Instantiates every variant for one attribute count (DV_ must be defined;
// 0 = generic kernel for any d <= 16).
#define KC_BOUND_DISPATCH(NAME, OBJNAME)                                                  \
  namespace kcb {                                                                        \
  kc_status NAME(int S, int NG, int KC, bool point, int skip, const BoundArgs &A, int grid,   \
                 size_t lds, hipStream_t st) {                                            \
    if (skip) return launch_ts<DV_>(S, NG, KC, point, A, grid, lds, st);                  \
    dim3 g(grid), b(WG);                                                                  \
    if (point) {                                                                          \
      KCB_PT_VARIANTS(KCB_PT_CASE)                                                        \
      return KC_EUNSUPPORTED;                                                             \
    }                                                                                     \
    if (KC > 0) {                                                                         \
      KCB_CAND_VARIANTS(KCB_CAND_CASE)                                                    \
      return KC_EUNSUPPORTED;                                                             \
    }                                                                                     \
    KCB_LB_VARIANTS(KCB_LB_CASE)                                                          \
    return KC_EUNSUPPORTED;                                                               \
  }                                                                                       \
  kc_status OBJNAME(const Obj64Args &A, int splits, size_t lds, hipStream_t st) {          \
    k_obj64<DV_><<<dim3(splits, A.n_sets), dim3(WG), lds, st>>>(A);                        \
    return KC_OK;                                                                         \
  }                                                                                       \
  }
