// kc_order.hip -- spatial (Morton) order of the active samples.
//
// The bound and tightening kernels give the same results for any order of the
// samples; in an order where consecutive samples are close, the samples a
// wavefront holds span a small box, so whole wavefronts settle their box tests
// at once and their branches agree. The driver applies this order once, after
// the root pass: Morton keys over the root box, with about 64 samples per key
// cell on average (at most 32 key bits), and a radix sort of (key, sample)
// pairs whose values carry the coordinates and the original id, so that the
// samples move with the sort's streaming passes instead of a random gather
// afterwards; the sorted pairs are then split back into rows.
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

// A sample travelling with its key: coordinates and original id.
template <int D>
struct SampleVal {
  float x[D];
  uint32_t id;
};

template <int D>
__global__ void k_keys_vals(KeyArgs A, const uint32_t *ids_in, SampleVal<D> *val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  const uint32_t qmax = (1u << A.bits) - 1u;
  uint32_t key = 0;
  SampleVal<D> v;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    v.x[a] = A.x[(int64_t)a * A.ld + i];
    const float t = (v.x[a] - A.lo[a]) * A.scale[a];
    uint32_t q = 0;
    if (t >= (float)qmax)
      q = qmax;
    else if (t > 0.f)  // false for NaN
      q = (uint32_t)t;
    for (int b = 0; b < A.bits; ++b) key |= ((q >> b) & 1u) << (b * D + a);
  }
  v.id = ids_in ? ids_in[i] : (uint32_t)i;
  A.key[i] = key;
  val[i] = v;
}

template <int D>
__global__ void k_unpack(const SampleVal<D> *val, int64_t n, float *y, int64_t ld_out,
                         uint32_t *ids_out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const SampleVal<D> v = val[j];
#pragma unroll
  for (int a = 0; a < D; ++a) y[(int64_t)a * ld_out + j] = v.x[a];
  ids_out[j] = v.id;
}

// Sort of (key, SampleVal<D>) pairs; false when d has no such path.
template <int D>
static kc_status sort_with_values(kc_handle *h, KeyArgs &A, const uint32_t *ids_in, int end_bit,
                                  float *x_out, uint32_t *ids_out, int64_t ld_out,
                                  hipStream_t st) {
  const int64_t n = A.n;
  using V = SampleVal<D>;
  hipcub::DoubleBuffer<uint32_t> keys(nullptr, nullptr);
  hipcub::DoubleBuffer<V> vals(nullptr, nullptr);
  size_t tmp_bytes = 0;
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, keys, vals, (int)n, 0, end_bit, st) !=
      hipSuccess)
    return kc_fail(h, KC_EDEVICE, "spatial order: sort size query");
  const size_t kb = ((size_t)n * 4 + 255) & ~(size_t)255;
  const size_t vb = ((size_t)n * sizeof(V) + 255) & ~(size_t)255;
  char *buf = nullptr;
  if (hipMalloc((void **)&buf, 2 * kb + 2 * vb + tmp_bytes + 256) != hipSuccess) {
    (void)hipGetLastError();
    return kc_fail(h, KC_ENOMEM, "spatial order: sort buffers");
  }
  keys = hipcub::DoubleBuffer<uint32_t>((uint32_t *)buf, (uint32_t *)(buf + kb));
  vals = hipcub::DoubleBuffer<V>((V *)(buf + 2 * kb), (V *)(buf + 2 * kb + vb));
  void *tmp = buf + 2 * kb + 2 * vb;
  A.key = keys.Current();
  const int T = 256;
  const int64_t blocks = (n + T - 1) / T;
  kc_status s = KC_OK;
  k_keys_vals<D><<<(unsigned)blocks, T, 0, st>>>(A, ids_in, vals.Current());
  s = kc_check_launch(h, "k_keys_vals");
  if (s == KC_OK &&
      hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, keys, vals, (int)n, 0, end_bit, st) !=
          hipSuccess)
    s = kc_fail(h, KC_EDEVICE, "spatial order: sort");
  if (s == KC_OK) {
    k_unpack<D><<<(unsigned)blocks, T, 0, st>>>(vals.Current(), n, x_out, ld_out, ids_out);
    s = kc_check_launch(h, "k_unpack");
  }
  (void)hipStreamSynchronize(st);
  (void)hipFree(buf);
  return s;
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
  // key bits: about 64 samples per key cell on average, whole radix digits of
  // 8 bits, at most 32 bits and 31 per attribute (so that 1u << bits stays
  // defined for d = 1)
  int lg = 0;
  while (lg < 40 && ((int64_t)1 << lg) < n) ++lg;
  int total = ((lg - 6 + 7) / 8) * 8;
  total = total < 8 ? 8 : (total > 32 ? 32 : total);
  A.bits = total / d;
  if (A.bits < 1) A.bits = 1;
  if (A.bits > 31) A.bits = 31;
  const float qmax = (float)((1u << A.bits) - 1u);
  for (int a = 0; a < d; ++a) {
    A.lo[a] = lo[a];
    const double w = (double)hi[a] - (double)lo[a];
    A.scale[a] = w > 0 ? (float)(qmax / w) : 0.f;
  }
  const int end_bit_v = A.bits * d;
  switch (d) {
    case 1: return sort_with_values<1>(h, A, ids_in, end_bit_v, x_out, ids_out, ld_out, st);
    case 2: return sort_with_values<2>(h, A, ids_in, end_bit_v, x_out, ids_out, ld_out, st);
    case 3: return sort_with_values<3>(h, A, ids_in, end_bit_v, x_out, ids_out, ld_out, st);
    case 4: return sort_with_values<4>(h, A, ids_in, end_bit_v, x_out, ids_out, ld_out, st);
    case 5: return sort_with_values<5>(h, A, ids_in, end_bit_v, x_out, ids_out, ld_out, st);
    case 6: return sort_with_values<6>(h, A, ids_in, end_bit_v, x_out, ids_out, ld_out, st);
    case 7: return sort_with_values<7>(h, A, ids_in, end_bit_v, x_out, ids_out, ld_out, st);
    case 8: return sort_with_values<8>(h, A, ids_in, end_bit_v, x_out, ids_out, ld_out, st);
    default: break;  // more attributes: sort (key, position), then gather
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
