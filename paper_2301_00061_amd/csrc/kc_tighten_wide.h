// kc_tighten_wide.h -- the tightening kernel with wavefront tile decisions
// over many nodes per workgroup (included by kc_tighten_impl.h; attribute
// counts 1..8, all boxes of a node in one chunk, no labels).
//
// Lane (jn, k) of every wavefront owns box k of node jn (NG << lg_kp <= 64):
// it classifies its box against each wavefront tile of samples (the tile's
// bounding box, with the per-sample operations in the same order, so a bound
// on the safe side of a threshold decides every sample alike) and keeps the
// box's aggregates in its own registers. What a tile settles folds into the
// owning lanes directly; the (tile, node) pairs it leaves open run the
// per-sample tests of Algorithms 3-4 and fold their per-box results with
// wavefront reductions. Without per-node register arrays, many nodes share
// one read of the samples.
#pragma once

namespace kct {

// CAP: registers limited to four wavefronts per SIMD (a grid of four
// workgroups per compute unit is then resident at once)
template <int D, int S, int NG, bool REFS, bool CAP>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(CAP ? 4 : 1))) void k_tighten_wide(TightenArgs A) {
  static_assert(D >= 1 && D <= 8, "tile decisions are compiled for 1..8 attributes");
  constexpr int DM = D;
  extern __shared__ float sm[];  // per node slot: boxes [k_max][2DM], refs' boxes, refs
  __shared__ NodeSlot s_node[NG];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int u = kcd::xcd_unit(blockIdx.x, gridDim.x);
  const int grp = u % A.n_groups, split = u / A.n_groups;  // one chunk of boxes
  const int m0 = grp * NG;
  stage_nodes<DM, NG, REFS>(A, m0, s_node, sm, D, tid);
  const int box_floats = A.k_max * 2 * DM;

  const int lg = A.lg_kp, KP = 1 << lg;
  const int cj = lane >> lg, ck = lane & (KP - 1);
  const int cjc = cj < NG ? cj : 0;
  const bool nvalid = cj < NG && m0 + cj < A.n_nodes;
  const int ccnt = nvalid ? s_node[cjc].cnt : 0;
  const bool cvalid = nvalid && ck < ccnt;
  const int sh = cj << lg;  // the lane's node segment in a ballot
  const uint64_t vm = ccnt >= 64 ? ~0ull : ((1ull << ccnt) - 1ull);
  const bool callref = REFS && nvalid && s_node[cjc].allref != 0;
  const int crc = REFS && cvalid ? s_node[cjc].rcnt[ck] : 0;
  const float *cbx = sm + cjc * A.node_floats + (cvalid ? ck : 0) * 2 * DM;
  const float *crbx = cbx + box_floats;
  const float *crf = sm + cjc * A.node_floats + 2 * box_floats + (REFS && cvalid ? s_node[cjc].rbeg[ck] : 0) * DM;
  uint64_t live = 0;  // bit jn: node jn exists
#pragma unroll
  for (int jn = 0; jn < NG; ++jn)
    if (m0 + jn < A.n_nodes) live |= 1ull << jn;

  // aggregates of box ck of node cj (valid lanes); nex of node cj in lane ck == 0
  float bmin[DM], bmax[DM], amin[DM], amax[DM];
#pragma unroll
  for (int a = 0; a < DM; ++a) {
    bmin[a] = amin[a] = INFINITY;
    bmax[a] = amax[a] = -INFINITY;
  }
  uint32_t nin = 0, nasg = 0, nex = 0;
  uint64_t far = 0;
  float fw = -1.f;  // at most the farthest folded distance of a sample assigned to the box

  const int64_t s_lo = (int64_t)split * A.span;
  const int64_t s_hi = min(A.n, s_lo + A.span);
  const int64_t lane_off = (int64_t)tid * S;
  for (int64_t base = s_lo + lane_off; base - lane_off < s_hi; base += (int64_t)WG * S) {
    const int64_t wb = base - lane_off + (int64_t)wave * 64 * S;
    if (wb >= s_hi) continue;  // no sample of this wavefront lies in the split (uniform)
    const uint32_t nval = (uint32_t)(s_hi - wb >= 64 * S ? 64 * S : s_hi - wb);
    // nodes whose chunk of samples the inside-only kernel took (uniform)
    uint64_t lightm = 0;
    if (A.light_map) {
#pragma unroll
      for (int jn = 0; jn < NG; ++jn)
        if (m0 + jn < A.n_nodes && A.light_map[(int64_t)(m0 + jn) * A.n_lchunks + wb / LCHUNK])
          lightm |= 1ull << jn;
    }
    const bool act = nvalid && !((lightm >> cjc) & 1ull);
    float xs[S][DM];
    const bool full = base + S <= s_hi;
#pragma unroll
    for (int a = 0; a < DM; ++a) {
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
      } else {
#pragma unroll
        for (int i = 0; i < S; ++i) xs[i][a] = (base + i < s_hi) ? p[i] : 0.f;
      }
    }
    float tlo[DM], thi[DM];
#pragma unroll
    for (int a = 0; a < DM; ++a) {
      float l = INFINITY, h = -INFINITY;
#pragma unroll
      for (int i = 0; i < S; ++i)
        if (base + i < s_hi) {
          l = fminf(l, xs[i][a]);
          h = fmaxf(h, xs[i][a]);
        }
      tlo[a] = __int_as_float(__builtin_amdgcn_readfirstlane(
          __float_as_int(kcd::fdec(kcd::wave_min_u32(kcd::ford(l))))));
      thi[a] = __int_as_float(__builtin_amdgcn_readfirstlane(
          __float_as_int(kcd::fdec(kcd::wave_max_u32(kcd::ford(h))))));
    }

    // Lane classification of box ck of node cj over the tile: center-based
    // exclusion of every / no sample, inside for every / no sample; with
    // refs, every sample within 4 alpha of every ref (near) or of none in
    // some ref (far), and likewise for alpha (the balls of S_+).
    bool c_out = false, c_keep = false, in_all = false, in_none = true;
    bool near_all = true, near_none = false, ball_all = true, ball_none = false;
    // whether a sample of the tile can change the box's aggregates as this
    // wavefront holds them: the assigned and S_+ bounding boxes (a value
    // inside both ends changes neither), the farthest assigned sample (a tile
    // wholly nearer the midpoint than a folded one cannot hold it)
    bool a_chg = false, b_chg = false, f_chg = false;
    float lm = 0.f, um = 0.f;
    if (cvalid) {
      float lb = 0.f, ub = 0.f;
      in_all = true;
      in_none = false;
#pragma unroll
      for (int a = 0; a < DM; ++a) {
        const float lo = cbx[2 * a], hi = cbx[2 * a + 1];
        const float g = fmaxf(fmaxf(lo - thi[a], tlo[a] - hi), 0.f);
        const float uu = fmaxf(fmaxf(lo - tlo[a], thi[a] - hi), 0.f);
        lb = (a == 0) ? g * g : __builtin_fmaf(g, g, lb);
        ub = (a == 0) ? uu * uu : __builtin_fmaf(uu, uu, ub);
        const float mid = 0.5f * (lo + hi);
        const float gm = fmaxf(fmaxf(mid - thi[a], tlo[a] - mid), 0.f);
        const float um2 = fmaxf(thi[a] - mid, mid - tlo[a]);
        lm = (a == 0) ? gm * gm : __builtin_fmaf(gm, gm, lm);
        um = (a == 0) ? um2 * um2 : __builtin_fmaf(um2, um2, um);
        in_all = in_all && lo <= tlo[a] && thi[a] <= hi;
        in_none = in_none || thi[a] < lo || tlo[a] > hi;
      }
      c_out = lb > A.t_center;
      c_keep = !(ub > A.t_center);
#pragma unroll
      for (int a = 0; a < DM; ++a) {
        a_chg = a_chg || tlo[a] < amin[a] || thi[a] > amax[a];
        b_chg = b_chg || tlo[a] < bmin[a] || thi[a] > bmax[a];
      }
      f_chg = !(um < fw);
      if (REFS && crc > 0) {
        // the refs' bounding box settles most tiles; else each ref
        float bn = 0.f, bx = 0.f;
#pragma unroll
        for (int a = 0; a < DM; ++a) {
          const float g = fmaxf(fmaxf(crbx[2 * a] - thi[a], tlo[a] - crbx[2 * a + 1]), 0.f);
          const float uu = fmaxf(thi[a] - crbx[2 * a], crbx[2 * a + 1] - tlo[a]);
          bn = (a == 0) ? g * g : __builtin_fmaf(g, g, bn);
          bx = (a == 0) ? uu * uu : __builtin_fmaf(uu, uu, bx);
        }
        const bool s_dec = !(bx > A.t_sample) || bn > A.t_sample;
        const bool b_dec = !(bx > A.t_ball) || bn > A.t_ball;
        if (s_dec && b_dec) {
          near_all = !(bx > A.t_sample);
          near_none = bn > A.t_sample;
          ball_all = !(bx > A.t_ball);
          ball_none = bn > A.t_ball;
        } else {
          for (int r = 0; r < crc; ++r) {
            const float *rr = crf + r * DM;
            float dn = 0.f, dx = 0.f;
#pragma unroll
            for (int a = 0; a < DM; ++a) {
              const float g = fmaxf(fmaxf(rr[a] - thi[a], tlo[a] - rr[a]), 0.f);
              const float uu = fmaxf(thi[a] - rr[a], rr[a] - tlo[a]);
              dn = (a == 0) ? g * g : __builtin_fmaf(g, g, dn);
              dx = (a == 0) ? uu * uu : __builtin_fmaf(uu, uu, dx);
            }
            near_all = near_all && !(dx > A.t_sample);
            near_none = near_none || dn > A.t_sample;
            ball_all = ball_all && !(dx > A.t_ball);
            ball_none = ball_none || dn > A.t_ball;
          }
        }
      }
    }
    const uint64_t b_out = __ballot(c_out), b_keep = __ballot(c_keep);
    const uint64_t b_achg = __ballot(a_chg), b_bchg = __ballot(b_chg), b_fchg = __ballot(f_chg);
    const uint64_t b_near = __ballot(near_all), b_nnone = __ballot(near_none);

    // The node's label over the tile (as the per-sample rule: every box but
    // one excluding the sample assigns it, every box excluding it drops it,
    // else the refs decide when each box has some), or unsettled.
    const uint64_t o = (b_out >> sh) & vm, kp = (b_keep >> sh) & vm;
    bool settled = (o | kp) == vm;
    const int n_out = __popcll(o);
    int lab = n_out == ccnt ? -2 : (n_out == ccnt - 1 ? __builtin_ctzll(vm & ~o) : -1);
    if (settled && lab == -1 && callref) {
      const uint64_t na = (b_near >> sh) & vm, nn = (b_nnone >> sh) & vm;
      if (__popcll(na) < 2) {
        if ((na | nn) != vm)
          settled = false;  // a box near some samples only: per sample
        else if (na)
          lab = __builtin_ctzll(na);
      }
    }
    if (!act) settled = true;

    // settled nodes: tile folds in the owning lanes
    bool far_open = false, sp_open = false;
    if (settled && act) {
      if (lab == -2 && ck == 0) nex += nval;
      if (cvalid && lab == ck) {
        nasg += nval;
#pragma unroll
        for (int a = 0; a < DM; ++a) {
          amin[a] = fminf(amin[a], tlo[a]);
          amax[a] = fmaxf(amax[a], thi[a]);
        }
        // an earlier tile of this box holds an assigned sample farther from
        // the midpoint than any sample of this one: its key cannot change
        far_open = !(um < fw);
        fw = fmaxf(fw, lm);
      }
      if (cvalid && !in_none) {
        // S_+: inside the box and within alpha of every ref of the box
        const bool balls = REFS && crc > 0;
        if (!(balls && ball_none)) {
          if (in_all && (!balls || ball_all)) {
            nin += nval;
#pragma unroll
            for (int a = 0; a < DM; ++a) {
              bmin[a] = fminf(bmin[a], tlo[a]);
              bmax[a] = fmaxf(bmax[a], thi[a]);
            }
          } else {
            sp_open = true;
          }
        }
      }
    }
    const uint64_t b_unset = __ballot(ck == 0 && !settled);
    const uint64_t b_far = __ballot(far_open), b_sp = __ballot(sp_open);
    uint64_t work = 0;
#pragma unroll
    for (int jn = 0; jn < NG; ++jn) {
      const uint64_t seg = KP >= 64 ? ~0ull : ((1ull << KP) - 1ull);
      if ((((b_far | b_sp) >> (jn << lg)) & seg) || ((b_unset >> (jn << lg)) & 1ull))
        work |= 1ull << jn;
    }
    work &= live & ~lightm;

    // the open (tile, node) work, per sample
    while (work) {
      const int jn = __builtin_ctzll(work);
      work &= work - 1;
      const NodeSlot &ns = s_node[jn];
      const int cnt = __builtin_amdgcn_readfirstlane(ns.cnt);
      const float *bx = sm + jn * A.node_floats;
      const float *rbx = bx + box_floats;
      const float *rf = rbx + box_floats;
      const bool unset = (b_unset >> (jn << lg)) & 1ull;
      int labs[S];
      if (unset) {
        // Center-based assignment (Lemma 1), then sample-based (Lemma 2)
        const bool allref = REFS && __builtin_amdgcn_readfirstlane(ns.allref) != 0;
        uint32_t nexl = 0;
#pragma unroll
        for (int i = 0; i < S; ++i) {
          int n_o = 0, keep = -1;
          for (int k = 0; k < cnt; ++k) {
            float acc = 0.f;
#pragma unroll
            for (int a = 0; a < DM; ++a) {
              const float t = xs[i][a] - kcd::med3(bx[k * 2 * DM + 2 * a], xs[i][a],
                                                   bx[k * 2 * DM + 2 * a + 1]);
              acc = (a == 0) ? t * t : __builtin_fmaf(t, t, acc);
            }
            const bool out = acc > A.t_center;
            n_o += out;
            keep = out ? keep : k;
          }
          int lb = n_o == cnt ? -2 : (n_o == cnt - 1 ? keep : -1);
          if (REFS && lb == -1 && allref) {
            int n_near = 0, rest_k = -1;
            for (int k = 0; k < cnt && n_near < 2; ++k) {
              const int rb = __builtin_amdgcn_readfirstlane(ns.rbeg[k]);
              const int rc = __builtin_amdgcn_readfirstlane(ns.rcnt[k]);
              if (all_refs_within(xs[i], rbx + k * 2 * DM, rf + rb * DM, rc, A.t_sample, D, DM)) {
                ++n_near;
                rest_k = k;
              }
            }
            if (n_near == 1) lb = rest_k;
          }
          if (base + i >= s_hi) lb = -3;
          nexl += lb == -2;
          labs[i] = lb;
        }
        const uint32_t e = kcd::wave_sum_u32(nexl);
        if (lane == (jn << lg)) nex += e;
      } else {
        const int lj = __shfl(lab, jn << lg);  // the node's settled label
#pragma unroll
        for (int i = 0; i < S; ++i) labs[i] = base + i < s_hi ? lj : -3;
      }
      for (int k = 0; k < cnt; ++k) {
        const int bit = (jn << lg) + k;
        const bool fo = (b_far >> bit) & 1ull, so = (b_sp >> bit) & 1ull;
        const bool owner = lane == bit;
        if (unset || fo) {
          // samples assigned to box k: count, bounding box (unsettled tiles;
          // settled ones folded the tile's) and the farthest from the midpoint
          float mid[DM];
#pragma unroll
          for (int a = 0; a < DM; ++a) mid[a] = 0.5f * (bx[k * 2 * DM + 2 * a] + bx[k * 2 * DM + 2 * a + 1]);
          uint32_t c = 0;
          float mn[DM], mx[DM];
#pragma unroll
          for (int a = 0; a < DM; ++a) {
            mn[a] = INFINITY;
            mx[a] = -INFINITY;
          }
          uint64_t key = 0;
#pragma unroll
          for (int i = 0; i < S; ++i) {
            if (labs[i] != k) continue;
            ++c;
            float dm = 0.f;
#pragma unroll
            for (int a = 0; a < DM; ++a) {
              mn[a] = fminf(mn[a], xs[i][a]);
              mx[a] = fmaxf(mx[a], xs[i][a]);
              const float w = xs[i][a] - mid[a];
              dm = (a == 0) ? w * w : __builtin_fmaf(w, w, dm);
            }
            const uint64_t kk = kcd::key_max(dm, (uint32_t)(base + i));
            key = kk > key ? kk : key;
          }
          if (fo || ((b_fchg >> bit) & 1ull)) {
            key = kcd::wave_max_u64(key);
            if (owner) {
              far = key > far ? key : far;
              if (key) fw = fmaxf(fw, __uint_as_float((uint32_t)(key >> 32)));
            }
          }
          if (unset) {
            const uint32_t cs = kcd::wave_sum_u32(c);
            if (owner) nasg += cs;
            if (cs && ((b_achg >> bit) & 1ull))
#pragma unroll
            for (int a = 0; a < DM; ++a) {
              const float v0 = kcd::fdec(kcd::wave_min_u32(kcd::ford(mn[a])));
              const float v1 = kcd::fdec(kcd::wave_max_u32(kcd::ford(mx[a])));
              if (owner) {
                amin[a] = fminf(amin[a], v0);
                amax[a] = fmaxf(amax[a], v1);
              }
            }
          }
        }
        if (unset || so) {
          // S_+^k: inside box k and within alpha of every ref of box k
          const int rb = __builtin_amdgcn_readfirstlane(ns.rbeg[k]);
          const int rc = REFS ? __builtin_amdgcn_readfirstlane(ns.rcnt[k]) : 0;
          uint32_t c = 0;
          float mn[DM], mx[DM];
#pragma unroll
          for (int a = 0; a < DM; ++a) {
            mn[a] = INFINITY;
            mx[a] = -INFINITY;
          }
#pragma unroll
          for (int i = 0; i < S; ++i) {
            bool in = base + i < s_hi;
#pragma unroll
            for (int a = 0; a < DM; ++a)
              in = in && bx[k * 2 * DM + 2 * a] <= xs[i][a] && xs[i][a] <= bx[k * 2 * DM + 2 * a + 1];
            if (REFS && in && rc > 0)
              in = all_refs_within(xs[i], rbx + k * 2 * DM, rf + rb * DM, rc, A.t_ball, D, DM);
            if (in) {
              ++c;
#pragma unroll
              for (int a = 0; a < DM; ++a) {
                mn[a] = fminf(mn[a], xs[i][a]);
                mx[a] = fmaxf(mx[a], xs[i][a]);
              }
            }
          }
          const uint32_t cs = kcd::wave_sum_u32(c);
          if (owner) nin += cs;
          if (cs && ((b_bchg >> bit) & 1ull)) {
#pragma unroll
            for (int a = 0; a < DM; ++a) {
              const float v0 = kcd::fdec(kcd::wave_min_u32(kcd::ford(mn[a])));
              const float v1 = kcd::fdec(kcd::wave_max_u32(kcd::ford(mx[a])));
              if (owner) {
                bmin[a] = fminf(bmin[a], v0);
                bmax[a] = fmaxf(bmax[a], v1);
              }
            }
          }
        }
      }
    }
  }

  // one atomic per value and owning lane
  if (cvalid) {
    const int64_t b = s_node[cj].b0 + ck;
    if (nin) atomicAdd(&A.n_in[b], nin);
    if (nasg) {
      atomicAdd(&A.n_asg[b], nasg);
      if (A.asg_far) atomicMax((unsigned long long *)&A.asg_far[b], (unsigned long long)far);
    }
#pragma unroll
    for (int a = 0; a < DM; ++a) {
      const int64_t o2 = b * D + a;
      if (nin) {
        atomicMin(&A.bb_lo[o2], kcd::ford(bmin[a]));
        atomicMax(&A.bb_hi[o2], kcd::ford(bmax[a]));
      }
      if (nasg) {
        atomicMin(&A.asg_min[o2], kcd::ford(amin[a]));
        atomicMax(&A.asg_max[o2], kcd::ford(amax[a]));
      }
    }
  }
  if (nvalid && ck == 0 && nex) atomicAdd(&A.n_excl[m0 + cj], nex);
}

template <int D>
inline bool launch_wide(int S, int NG, bool cap, bool refs, const TightenArgs &A, int grid,
                        size_t lds, hipStream_t st) {
  if constexpr (D >= 1 && D <= 8) {
#define KCT_WIDE(SV, NGV)                                                        \
  if (S == SV && NG == NGV) {                                                   \
    if (cap && SV <= 8) {                                                       \
      if (refs)                                                                 \
        k_tighten_wide<D, SV, NGV, true, SV <= 8><<<grid, WG, lds, st>>>(A);    \
      else                                                                      \
        k_tighten_wide<D, SV, NGV, false, SV <= 8><<<grid, WG, lds, st>>>(A);   \
    } else if (refs) {                                                          \
      k_tighten_wide<D, SV, NGV, true, false><<<grid, WG, lds, st>>>(A);        \
    } else {                                                                    \
      k_tighten_wide<D, SV, NGV, false, false><<<grid, WG, lds, st>>>(A);       \
    }                                                                           \
    return true;                                                                \
  }
    KCT_WIDE_VARIANTS(KCT_WIDE)
#undef KCT_WIDE
  }
  return false;
}

}  // namespace kct
