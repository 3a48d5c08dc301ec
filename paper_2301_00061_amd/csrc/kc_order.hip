// kc_order.hip -- spatial (Morton) order of the active samples.
//
// The bound and tightening kernels give the same results for any order of the
// samples; in an order where consecutive samples are close, the 256 samples a
// wavefront holds span a small box, so whole wavefronts settle their box tests
// at once and their branches agree. The driver applies this order once, after
// the root pass: keys from the root box, a radix sort of (key, position), and
// a gather that writes the reordered coordinates and the map to original ids.
#include <hipcub/hipcub.hpp>

#include "kc_internal.h"

namespace kcm {

constexpr int MAXD = 16;

struct KeyArgs {
  const float *x;
  int64_t n, ld;
  int d, bits;
  float lo[MAXD], scale[MAXD];
  uint32_t *key, *pos;
};

// Quantize each attribute to `bits` bits over the root box and interleave
// them (bit b of attribute a goes to bit b*d + a).
__global__ void k_keys(KeyArgs A) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  const uint32_t qmax = (1u << A.bits) - 1u;
  uint32_t key = 0;
  for (int a = 0; a < A.d; ++a) {
    const float v = (A.x[(int64_t)a * A.ld + i] - A.lo[a]) * A.scale[a];
    uint32_t q = 0;
    if (v >= (float)qmax)
      q = qmax;
    else if (v > 0.f)  // false for NaN
      q = (uint32_t)v;
    for (int b = 0; b < A.bits; ++b) key |= ((q >> b) & 1u) << (b * A.d + a);
  }
  A.key[i] = key;
  A.pos[i] = (uint32_t)i;
}

// y[a][j] = x[a][perm[j]]; ids_out[j] = ids_in ? ids_in[perm[j]] : perm[j].
__global__ void k_permute(const float *x, int64_t ld_in, int d, const uint32_t *perm,
                          const uint32_t *ids_in, int64_t n, float *y, int64_t ld_out,
                          uint32_t *ids_out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const uint32_t p = perm[j];
  for (int a = 0; a < d; ++a) y[(int64_t)a * ld_out + j] = x[(int64_t)a * ld_in + p];
  ids_out[j] = ids_in ? ids_in[p] : p;
}

}  // namespace kcm

kc_status kc_spatial_order(kc_handle *h, const kc_points *in, const uint32_t *ids_in,
                           const float *lo, const float *hi, float *x_out, uint32_t *ids_out,
                           int64_t ld_out, hipStream_t st) {
  using namespace kcm;
  const int64_t n = in->n;
  const int d = in->d;
  if (n < 1 || d < 1 || d > MAXD || ld_out < n) return kc_fail(h, KC_EINVAL, "spatial order: bad sizes");
  KeyArgs A{};
  A.x = in->x;
  A.n = n;
  A.ld = in->ld;
  A.d = d;
  // at most 31 bits per attribute, so that 1u << bits stays defined (d = 1)
  A.bits = 32 / d < 31 ? 32 / d : 31;
  const float qmax = (float)((1u << A.bits) - 1u);
  for (int a = 0; a < d; ++a) {
    A.lo[a] = lo[a];
    const double w = (double)hi[a] - (double)lo[a];
    A.scale[a] = w > 0 ? (float)(qmax / w) : 0.f;
  }
  // keys and positions, double-buffered for the sort, plus its temporary
  uint32_t *buf = nullptr;
  void *tmp = nullptr;
  size_t tmp_bytes = 0;
  const int end_bit = A.bits * d;
  hipcub::DoubleBuffer<uint32_t> keys(nullptr, nullptr), vals(nullptr, nullptr);
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, keys, vals, (int)n, 0, end_bit, st) !=
      hipSuccess)
    return kc_fail(h, KC_EDEVICE, "spatial order: sort size query");
  if (hipMalloc((void **)&buf, (size_t)n * 16) != hipSuccess) {
    (void)hipGetLastError();
    return kc_fail(h, KC_ENOMEM, "spatial order: key buffers");
  }
  if (hipMalloc(&tmp, tmp_bytes + 256) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(buf);
    return kc_fail(h, KC_ENOMEM, "spatial order: sort temporary");
  }
  keys = hipcub::DoubleBuffer<uint32_t>(buf, buf + n);
  vals = hipcub::DoubleBuffer<uint32_t>(buf + 2 * n, buf + 3 * n);
  A.key = keys.Current();
  A.pos = vals.Current();
  const int T = 256;
  const int64_t blocks = (n + T - 1) / T;
  kc_status s = KC_OK;
  k_keys<<<(unsigned)blocks, T, 0, st>>>(A);
  s = kc_check_launch(h, "k_keys");
  if (s == KC_OK &&
      hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, keys, vals, (int)n, 0, end_bit, st) !=
          hipSuccess)
    s = kc_fail(h, KC_EDEVICE, "spatial order: sort");
  if (s == KC_OK) {
    k_permute<<<(unsigned)blocks, T, 0, st>>>(in->x, in->ld, d, vals.Current(), ids_in, n, x_out,
                                              ld_out, ids_out);
    s = kc_check_launch(h, "k_permute");
  }
  (void)hipStreamSynchronize(st);
  (void)hipFree(tmp);
  (void)hipFree(buf);
  return s;
}
