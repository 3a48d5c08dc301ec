// kc_bound_wide.h -- the bound kernel with wavefront tile decisions over many
// nodes per workgroup (included by kc_bound_impl.h; attribute counts 1..8).
//
// A workgroup owns NG nodes (NG << lg_kp <= 64: one (node, box) pair per lane
// for the tile decisions) and one split of the samples. Per wavefront tile
// (64 * S consecutive samples) the lanes bound every box of every node over
// the tile's bounding box at once; a node whose tile the bounds settle skips
// it. Only the (tile, node) pairs left open are evaluated per sample, and
// their results are folded with wavefront reductions into per-wavefront
// running keys in LDS. Without per-node registers, many nodes share one read
// of the samples, which is what bounds a launch with few open tiles.
#pragma once

namespace kcb {

template <int D, int S, int NG, int KC, bool POINT>
__global__ __launch_bounds__(WG) void k_bound_wide(BoundArgs A) {
  static_assert(D >= 1 && D <= 8, "tile decisions are compiled for 1..8 attributes");
  constexpr int DM = D;
  extern __shared__ float smem[];  // [NG][k_max][DM] interleaved (lo, hi)
  __shared__ int s_beg[NG], s_cnt[NG];
  __shared__ uint64_t s_key[NWAVE][NG];
  __shared__ uint64_t s_cand[NWAVE][KC > 0 ? NG * KC : 1];

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
  __shared__ int s_dead0[NG];
  for (int i = tid; i < NWAVE * NG; i += WG) s_key[i / NG][i % NG] = 0ull;
  if constexpr (KC > 0)
    for (int i = tid; i < NWAVE * NG * KC; i += WG) s_cand[i / (NG * KC)][i % (NG * KC)] = ~0ull;
  __syncthreads();
  if (tid < NG) {
    // screening with a floor above the cut: the set cannot improve the
    // incumbent, and the lowered floor is a value it reaches -- reported
    // with no sample (index 0xffffffff), no tile evaluated
    int dead0 = 0;
    if (POINT && A.floor && A.dead && m0 + tid < A.n_nodes) {
      const double f = A.floor[m0 + tid] * (1.0 - A.frel) - A.fabs_;
      float ff = (float)f;
      if ((double)ff > f) ff = nextafterf(ff, -INFINITY);
      if (ff > A.cut) {
        dead0 = 1;
        if (split == 0) s_key[0][tid] = kcd::key_max(ff, 0xffffffffu);
      }
    }
    s_dead0[tid] = dead0;
  }
  const int per_node = A.k_max * 2 * DM;
  for (int i = tid; i < NG * A.k_max * DM; i += WG) {
    const int jn = i / (A.k_max * DM);
    const int r = i - jn * A.k_max * DM;
    const int k = r / DM, a = r - k * DM;
    float l = 0.0f, h = 0.0f;
    if (k < s_cnt[jn]) {
      const int64_t b = s_beg[jn] + k;
      l = A.lo[b * D + a];
      h = POINT ? l : A.hi[b * D + a];
    }
    smem[jn * per_node + k * 2 * DM + 2 * a] = l;
    smem[jn * per_node + k * 2 * DM + 2 * a + 1] = h;
  }
  __syncthreads();

  // Lane (jn, k) = (lane >> lg, lane & (KP - 1)) holds node jn's tile state:
  // Wl, a value the node's maximum over the tiles this wavefront folded has
  // reached (at a lower index than any later tile of the wavefront), cwl, a
  // distance to box k's midpoint that a sample inside box k folded here does
  // not exceed; Wg / cwg the values any wavefront published (at any index).
  const int lg = A.lg_kp, KP = 1 << lg;
  const int cj = lane >> lg, ck = lane & (KP - 1);
  const bool cvalid = cj < NG && m0 + cj < A.n_nodes && ck < s_cnt[cj < NG ? cj : 0];
  float Wl = -1.0f, cwl = INFINITY, Wg = -1.0f, cwg = INFINITY, Wpub = -1.0f, cpub = INFINITY;
  if (POINT && A.floor && cvalid) {
    // the set's float32 maximum is at least floor (1 - frel) - fabs
    const double f = A.floor[m0 + cj] * (1.0 - A.frel) - A.fabs_;
    float ff = (float)f;
    if ((double)ff > f) ff = nextafterf(ff, -INFINITY);
    Wg = fmaxf(Wg, ff);
  }
  uint64_t deadm = __ballot(lane < NG && s_dead0[lane < NG ? lane : 0] != 0);  // screening
  if constexpr (POINT) {
    // the witness sample of each set, with the per-sample operations: a
    // value above the cut settles the set there (wavefront 0 folds its key)
    if (A.wit_x && A.dead) {
      float v = INFINITY;
      int64_t wid = -1;
      if (cvalid) {
        wid = A.wit_id[m0 + cj];
        if (wid >= 0 && wid < A.n) {
          const float *B = smem + cj * per_node + ck * 2 * DM;
          const float *wx = A.wit_x + (int64_t)(m0 + cj) * D;
          float acc = 0.f;
#pragma unroll
          for (int a = 0; a < DM; ++a) {
            const float t = wx[a] - B[2 * a];
            acc = (a == 0) ? t * t : __builtin_fmaf(t, t, acc);
          }
          v = acc;
        }
      }
      v = kcd::group_min(v, KP);
      const bool kill = cvalid && ck == 0 && wid >= 0 && wid < A.n && v > A.cut;
      const uint64_t km = __ballot(kill);
#pragma unroll
      for (int jn = 0; jn < NG; ++jn)
        if ((km >> (jn << lg)) & 1ull) deadm |= 1ull << jn;
      if (kill && wave == 0) {
        const uint64_t key = kcd::key_max(v, (uint32_t)wid);
        if (key > s_key[0][cj]) s_key[0][cj] = key;
      }
    }
  }
  uint64_t live = 0;   // bit jn: node jn exists
#pragma unroll
  for (int jn = 0; jn < NG; ++jn)
    if (m0 + jn < A.n_nodes) live |= 1ull << jn;
  int tick = 0;

  const int64_t s_lo = (int64_t)split * A.span;
  const int64_t s_hi = min(A.n, s_lo + A.span);
  const int64_t lane_off = (int64_t)tid * S;
  // a lane's S consecutive samples from base (zeros past the split's end)
  auto load = [&](float (&xv)[DM][S], int64_t base) {
    const bool full = base + S <= s_hi;
#pragma unroll
    for (int a = 0; a < DM; ++a) {
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
    }
  };
  // the next tile's samples are requested before the current tile is
  // processed, so their latency overlaps its decisions and evaluations
  float xn[DM][S];
  if (s_lo < s_hi) load(xn, s_lo + lane_off);
  for (int64_t base = s_lo + lane_off; base - lane_off < s_hi; base += (int64_t)WG * S) {
    float xv[DM][S];
#pragma unroll
    for (int a = 0; a < DM; ++a)
#pragma unroll
      for (int i = 0; i < S; ++i) xv[a][i] = xn[a][i];
    if (base - lane_off + (int64_t)WG * S < s_hi) load(xn, base + (int64_t)WG * S);
    const bool refresh = (tick++ & 15) == 0;
    const int64_t wb = base - lane_off + (int64_t)wave * 64 * S;
    if (wb >= s_hi) continue;  // no sample of this wavefront lies in the split (uniform)
    if (POINT && !(live & ~deadm)) break;  // every set of the workgroup settled (uniform)
    float tlo[DM], thi[DM];
#pragma unroll
    for (int a = 0; a < DM; ++a) {
      float l = INFINITY, h = -INFINITY;
#pragma unroll
      for (int i = 0; i < S; ++i)
        if (base + i < s_hi) {
          l = fminf(l, xv[a][i]);
          h = fmaxf(h, xv[a][i]);
        }
      tlo[a] = __int_as_float(__builtin_amdgcn_readfirstlane(
          __float_as_int(kcd::fdec(kcd::wave_min_u32(kcd::ford(l))))));
      thi[a] = __int_as_float(__builtin_amdgcn_readfirstlane(
          __float_as_int(kcd::fdec(kcd::wave_max_u32(kcd::ford(h))))));
    }

    // share the tile state with the other wavefronts (every 16th tile);
    // every value stored was reached by some wavefront and they only move one
    // way, so a stale read is still a valid, weaker, bound
    if (A.gW && refresh && cvalid) {
      if (ck == 0) {
        uint32_t *gw = A.gW + m0 + cj;
        const uint32_t gv = Wl > Wpub ? atomicMax(gw, kcd::ford(Wl))
                                      : __hip_atomic_load(gw, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_WORKGROUP);
        Wpub = fmaxf(Wpub, Wl);
        Wg = fmaxf(Wg, kcd::fdec(gv));
      }
      if constexpr (KC > 0) {
        uint32_t *gc = A.gC + s_beg[cj] + ck;
        const uint32_t gv = cwl < cpub ? atomicMin(gc, kcd::ford(cwl))
                                       : __hip_atomic_load(gc, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_WORKGROUP);
        cpub = fminf(cpub, cwl);
        cwg = fminf(cwg, kcd::fdec(gv));
      }
    }
    if constexpr (POINT) {
      if (A.dead && refresh) {
        uint32_t f = 0;
        if (lane < NG && m0 + lane < A.n_nodes)
          f = __hip_atomic_load(A.dead + m0 + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        deadm |= __ballot(f != 0u);
      }
    }

    // Tile decisions: every sample's min_k of node jn lies in [lb_t, ub_t]
    // (the per-sample operations in the same order on the tile's extreme
    // coordinates; float32 rounding is monotone). ub_t <= Wl, or ub_t < Wg:
    // the tile cannot raise the node's maximum nor hold the lowest index
    // attaining it. With candidates, box k cannot get its candidate from a
    // tile it misses or whose whole range lies farther from its midpoint than
    // cwl (ties go to the lower index already folded) or cwg.
    float lbk = INFINITY, ubk = INFINITY;
    bool cskip = true;
    if (cvalid) {
      const float *B = smem + cj * per_node + ck * 2 * DM;
      float lb = 0.f, ub = 0.f, lm = 0.f, um = 0.f;
      bool ia = true, inn = false;
#pragma unroll
      for (int a = 0; a < DM; ++a) {
        const float l = B[2 * a], h = POINT ? l : B[2 * a + 1];
        const float gl = fmaxf(fmaxf(l - thi[a], tlo[a] - h), 0.f);
        const float ul = fmaxf(fmaxf(l - tlo[a], thi[a] - h), 0.f);
        lb = (a == 0) ? gl * gl : __builtin_fmaf(gl, gl, lb);
        ub = (a == 0) ? ul * ul : __builtin_fmaf(ul, ul, ub);
        if constexpr (KC > 0) {
          const float mid = 0.5f * (l + h);
          const float gm = fmaxf(fmaxf(mid - thi[a], tlo[a] - mid), 0.f);
          const float um2 = fmaxf(thi[a] - mid, mid - tlo[a]);
          lm = (a == 0) ? gm * gm : __builtin_fmaf(gm, gm, lm);
          um = (a == 0) ? um2 * um2 : __builtin_fmaf(um2, um2, um);
          ia = ia && l <= tlo[a] && thi[a] <= h;
          inn = inn || thi[a] < l || tlo[a] > h;
        }
      }
      lbk = lb;
      ubk = ub;
      if constexpr (KC > 0) {
        cskip = inn || lm >= cwl || lm > cwg;
        if (ia) cwl = fminf(cwl, um);
      }
    }
    lbk = kcd::group_min(lbk, KP);
    ubk = kcd::group_min(ubk, KP);
    bool ns = ubk <= Wl || ubk < Wg;
    Wl = fmaxf(Wl, lbk);
    if constexpr (KC > 0) {
      const uint64_t seg = KP >= 64 ? ~0ull : ((1ull << KP) - 1ull);
      ns = ns && ((__ballot(!cskip) >> (cj << lg)) & seg) == 0;
    }
    const uint64_t skipm = __ballot(ck == 0 && ns);
    uint64_t open = 0;
#pragma unroll
    for (int jn = 0; jn < NG; ++jn)
      if (!((skipm >> (jn << lg)) & 1ull)) open |= 1ull << jn;
    open &= live & ~deadm;

    // the open (tile, node) pairs, per sample
    while (open) {
      const int jn = __builtin_ctzll(open);
      open &= open - 1;
      const float *bx = smem + jn * per_node;
      const int cnt = s_cnt[jn];
      float best[S];
#pragma unroll
      for (int i = 0; i < S; ++i) best[i] = INFINITY;
      for (int k = 0; k < cnt; ++k) {
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
            const float c = POINT ? l[a] : kcd::med3(l[a], xv[a][i], h[a]);
            if constexpr (KC > 0) in[i] = in[i] && (c == xv[a][i]);
            const float t = xv[a][i] - c;
            acc = (a == 0) ? t * t : __builtin_fmaf(t, t, acc);
          }
          best[i] = fminf(best[i], acc);
        }
        if constexpr (KC > 0) {
          // the candidate of box k: the sample inside it nearest its
          // midpoint, lowest index on ties
          bool any = false;
#pragma unroll
          for (int i = 0; i < S; ++i) any = any || in[i];
          if (__ballot(any)) {
            uint64_t ckey = ~0ull;
#pragma unroll
            for (int i = 0; i < S; ++i) {
              float dm = 0.0f;
#pragma unroll
              for (int a = 0; a < DM; ++a) {
                const float w = xv[a][i] - 0.5f * (l[a] + h[a]);
                dm = (a == 0) ? w * w : __builtin_fmaf(w, w, dm);
              }
              const uint64_t kk = in[i] ? kcd::key_min(dm, (uint32_t)(base + i)) : ~0ull;
              ckey = kk < ckey ? kk : ckey;
            }
            ckey = kcd::wave_min_u64(ckey);
            if (lane == 0 && ckey < s_cand[wave][jn * KC + k]) s_cand[wave][jn * KC + k] = ckey;
            if (lane == (jn << lg) + k) cwl = fminf(cwl, __uint_as_float((uint32_t)(ckey >> 32)));
          }
        }
      }
      uint64_t key = 0ull;
#pragma unroll
      for (int i = 0; i < S; ++i)
        if (base + i < s_hi) {
          const uint64_t kk = kcd::key_max(best[i], (uint32_t)(base + i));
          key = kk > key ? kk : key;
        }
      key = kcd::wave_max_u64(key);
      if (lane == 0 && key > s_key[wave][jn]) s_key[wave][jn] = key;
      const float tv = key ? __uint_as_float((uint32_t)(key >> 32)) : -1.0f;
      if (cj == jn) Wl = fmaxf(Wl, tv);  // reached in this tile: lower index than later tiles
      if constexpr (POINT) {
        // screening: a value above the cut is folded; the set stops here and,
        // through dead[], in the other workgroups
        if (A.dead && tv > A.cut) {
          deadm |= 1ull << jn;
          if (lane == 0)
            __hip_atomic_store(A.dead + m0 + jn, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
  }
  __syncthreads();
  if (tid < NG && m0 + tid < A.n_nodes) {
    uint64_t key = s_key[0][tid];
#pragma unroll
    for (int w = 1; w < NWAVE; ++w) key = s_key[w][tid] > key ? s_key[w][tid] : key;
    A.part_key[(int64_t)split * A.n_nodes + m0 + tid] = key;
  }
  if constexpr (KC > 0) {
    for (int i = tid; i < NG * KC; i += WG) {
      const int jn = i / KC, k = i - jn * KC;
      if (m0 + jn < A.n_nodes && k < s_cnt[jn]) {
        uint64_t ck2 = s_cand[0][i];
#pragma unroll
        for (int w = 1; w < NWAVE; ++w) ck2 = s_cand[w][i] < ck2 ? s_cand[w][i] : ck2;
        A.part_cand[(int64_t)split * A.n_boxes + s_beg[jn] + k] = ck2;
      }
    }
  }
}

}  // namespace kcb
