// kc_util.hip -- small device helpers used by the host driver.
#include "kc_internal.h"

// Gathers the coordinates of `count` samples (active indices ids[i]) into
// out[i][d]; orig[i] receives idx_map[ids[i]] (or ids[i] without a map).
__global__ void k_gather(const float *x, int64_t ld, int d, int64_t n, const int64_t *ids,
                         int count, const uint32_t *idx_map, float *out, int64_t *orig) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  int64_t s = ids[i];
  if (s < 0 || s >= n) s = 0;  // callers pass valid ids; never read out of range
  for (int a = 0; a < d; ++a) out[(int64_t)i * d + a] = x[(int64_t)a * ld + s];
  if (orig) orig[i] = idx_map ? (int64_t)idx_map[s] : s;
}

kc_status kc_gather(kc_handle *h, const kc_points *p, const int64_t *ids, int count,
                    const uint32_t *idx_map, float *out, int64_t *orig, hipStream_t st) {
  if (count <= 0) return KC_OK;
  k_gather<<<(count + 255) / 256, 256, 0, st>>>(p->x, p->ld, p->d, p->n, ids, count, idx_map, out,
                                                orig);
  return kc_check_launch(h, "k_gather");
}
