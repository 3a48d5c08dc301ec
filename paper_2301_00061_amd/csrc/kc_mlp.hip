// kc_mlp.hip -- the branching network: a 32-64-64-64-1 ReLU perceptron that
// scores (cluster, attribute) split candidates. bf16 weights and inputs,
// float32 accumulation; hidden activations stay float32.
//
// forward   one lane per row; the weights (as float32) live in LDS and are
//           read by all lanes at the same address (broadcast).
// backward  phase 1, one lane per row: the gradients of the three hidden
//           layers' pre-activations; phase 2, one lane per parameter and row
//           chunk: sums over the chunk's rows; phase 3 adds the chunks in a
//           fixed order. No float atomics, so gradients are reproducible.
// loss      softmax cross-entropy over the rows of each group, mean over
//           groups, reduced in a fixed order by one workgroup.
// adam      elementwise on the float32 master copy, then round-to-nearest-even
//           to bf16.
#include <cmath>

#include "kc_device.h"
#include "kc_internal.h"

namespace kcm {

constexpr int NI = KC_MLP_IN, NH = KC_MLP_HID, NP = KC_MLP_PARAMS;
// offsets of the parameter blocks
constexpr int W1 = 0, B1 = W1 + NH * NI, W2 = B1 + NH, B2 = W2 + NH * NH, W3 = B2 + NH,
              B3 = W3 + NH * NH, W4 = B3 + NH, B4 = W4 + NH;
static_assert(B4 + 1 == NP, "parameter layout");

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);  // NaN
  const uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(r >> 16);
}

__device__ __forceinline__ void load_weights(const uint16_t *w, float *sw) {
  for (int i = threadIdx.x; i < NP; i += blockDim.x) sw[i] = bf16_to_f32(w[i]);
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_mlp_forward(const uint16_t *w, const float *feat, int64_t rows,
                                                     float *score, float *act) {
  extern __shared__ float sw[];
  load_weights(w, sw);
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  float x[NI], h[NH], g[NH];
#pragma unroll
  for (int i = 0; i < NI; ++i) x[i] = bf16_to_f32(f32_to_bf16(feat[r * NI + i]));
#pragma unroll 4
  for (int j = 0; j < NH; ++j) {
    float s = sw[B1 + j];
#pragma unroll
    for (int i = 0; i < NI; ++i) s = __builtin_fmaf(sw[W1 + j * NI + i], x[i], s);
    h[j] = fmaxf(s, 0.f);
  }
#pragma unroll 4
  for (int j = 0; j < NH; ++j) {
    float s = sw[B2 + j];
#pragma unroll
    for (int i = 0; i < NH; ++i) s = __builtin_fmaf(sw[W2 + j * NH + i], h[i], s);
    g[j] = fmaxf(s, 0.f);
  }
  if (act) {
    for (int j = 0; j < NH; ++j) act[r * 3 * NH + j] = h[j];
    for (int j = 0; j < NH; ++j) act[r * 3 * NH + NH + j] = g[j];
  }
#pragma unroll 4
  for (int j = 0; j < NH; ++j) {
    float s = sw[B3 + j];
#pragma unroll
    for (int i = 0; i < NH; ++i) s = __builtin_fmaf(sw[W3 + j * NH + i], g[i], s);
    h[j] = fmaxf(s, 0.f);
  }
  if (act)
    for (int j = 0; j < NH; ++j) act[r * 3 * NH + 2 * NH + j] = h[j];
  float s = sw[B4];
#pragma unroll
  for (int i = 0; i < NH; ++i) s = __builtin_fmaf(sw[W4 + i], h[i], s);
  score[r] = s;
}

// Phase 1: per row, the gradients of the pre-activations of layers 3, 2, 1
// (layer 4's is dscore itself), written to grad[r][192] as (g1, g2, g3).
__global__ __launch_bounds__(256) void k_mlp_back_rows(const uint16_t *w, const float *act,
                                                       const float *dscore, int64_t rows,
                                                       float *grad) {
  extern __shared__ float sw[];
  load_weights(w, sw);
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const float *h1 = act + r * 3 * NH, *h2 = h1 + NH, *h3 = h2 + NH;
  const float d4 = dscore[r];
  float g3[NH], g2[NH];
#pragma unroll
  for (int j = 0; j < NH; ++j) g3[j] = h3[j] > 0.f ? d4 * sw[W4 + j] : 0.f;
#pragma unroll 4
  for (int i = 0; i < NH; ++i) {
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < NH; ++j) s = __builtin_fmaf(g3[j], sw[W3 + j * NH + i], s);
    g2[i] = h2[i] > 0.f ? s : 0.f;
  }
  float *out = grad + r * 3 * NH;
  for (int j = 0; j < NH; ++j) out[NH + j] = g2[j];
  for (int j = 0; j < NH; ++j) out[2 * NH + j] = g3[j];
#pragma unroll 4
  for (int i = 0; i < NH; ++i) {
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < NH; ++j) s = __builtin_fmaf(g2[j], sw[W2 + j * NH + i], s);
    out[i] = h1[i] > 0.f ? s : 0.f;
  }
}

// Phase 2: one lane per parameter; rows [c*chunk, (c+1)*chunk) of chunk c.
__global__ __launch_bounds__(256) void k_mlp_back_params(const float *feat, const float *act,
                                                         const float *grad, const float *dscore,
                                                         int64_t rows, int64_t chunk,
                                                         float *part) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (p >= NP) return;
  const int64_t r0 = (int64_t)c * chunk;
  const int64_t r1 = min(rows, r0 + chunk);
  // parameter p = (layer, out j, in i) or a bias
  int gsel, gj, isel, ii;  // gradient row offset, input kind / index
  if (p < B1) {
    gsel = 0; gj = (p - W1) / NI; isel = 0; ii = (p - W1) % NI;
  } else if (p < W2) {
    gsel = 0; gj = p - B1; isel = -1; ii = 0;
  } else if (p < B2) {
    gsel = 1; gj = (p - W2) / NH; isel = 1; ii = (p - W2) % NH;
  } else if (p < W3) {
    gsel = 1; gj = p - B2; isel = -1; ii = 0;
  } else if (p < B3) {
    gsel = 2; gj = (p - W3) / NH; isel = 2; ii = (p - W3) % NH;
  } else if (p < W4) {
    gsel = 2; gj = p - B3; isel = -1; ii = 0;
  } else if (p < B4) {
    gsel = 3; gj = 0; isel = 3; ii = p - W4;
  } else {
    gsel = 3; gj = 0; isel = -1; ii = 0;
  }
  float s = 0.f;
  for (int64_t r = r0; r < r1; ++r) {
    const float gv = gsel == 3 ? dscore[r] : grad[r * 3 * NH + gsel * NH + gj];
    float in = 1.f;
    if (isel == 0)
      in = bf16_to_f32(f32_to_bf16(feat[r * NI + ii]));
    else if (isel > 0)
      in = act[r * 3 * NH + (isel - 1) * NH + ii];
    s = __builtin_fmaf(gv, in, s);
  }
  part[(int64_t)c * NP + p] = s;
}

__global__ void k_mlp_back_sum(const float *part, int n_chunks, float *dw) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NP) return;
  float s = 0.f;
  for (int c = 0; c < n_chunks; ++c) s += part[(int64_t)c * NP + p];
  dw[p] = s;
}

__global__ __launch_bounds__(256) void k_mlp_loss(const float *score, const int32_t *grp_off,
                                                  const int32_t *target, int n_groups, int64_t rows,
                                                  float *dscore, float *loss) {
  __shared__ float sl[256];
  // rows outside every group get a zero gradient
  for (int64_t r = threadIdx.x; r < rows; r += blockDim.x) dscore[r] = 0.f;
  __syncthreads();
  float acc = 0.f;
  const float inv = 1.f / (float)(n_groups > 0 ? n_groups : 1);
  for (int g = threadIdx.x; g < n_groups; g += blockDim.x) {
    int64_t a = grp_off[g], b = grp_off[g + 1];
    a = a < 0 ? 0 : (a > rows ? rows : a);
    b = b < a ? a : (b > rows ? rows : b);
    if (b <= a) continue;
    float m = -INFINITY;
    for (int64_t r = a; r < b; ++r) m = fmaxf(m, score[r]);
    float z = 0.f;
    for (int64_t r = a; r < b; ++r) z += expf(score[r] - m);
    int64_t t = a + target[g];
    if (t < a || t >= b) t = a;
    acc += -(score[t] - m - logf(z));
    for (int64_t r = a; r < b; ++r) {
      float p = expf(score[r] - m) / z;
      if (r == t) p -= 1.f;
      dscore[r] = p * inv;
    }
  }
  sl[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int i = 0; i < (int)blockDim.x; ++i) s += sl[i];
    loss[0] = s * inv;
  }
}

__global__ void k_mlp_adam(float *w32, uint16_t *wb, const float *g, float *m, float *v, float c1,
                           float c2, float lr) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NP) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float gi = g[p];
  const float mi = b1 * m[p] + (1.f - b1) * gi;
  const float vi = b2 * v[p] + (1.f - b2) * gi * gi;
  m[p] = mi;
  v[p] = vi;
  const float wi = w32[p] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w32[p] = wi;
  wb[p] = f32_to_bf16(wi);
}

}  // namespace kcm

using namespace kcm;

extern "C" kc_status kc_mlp_forward(kc_handle *h, const uint16_t *w_bf16, const float *feat,
                                    int64_t rows, float *score, float *act, void *stream) {
  return kc_guard(h, [&]() -> kc_status {
    if (!h) return KC_EINVAL;
    KC_RETURN_IF(!w_bf16 || !feat || !score, h, KC_EINVAL, "w / feat / score is NULL");
    KC_RETURN_IF(rows < 0, h, KC_EINVAL, "rows < 0");
    if (rows == 0) return KC_OK;
    const int64_t nb = (rows + 255) / 256;
    KC_RETURN_IF(nb > 0x7fffffff, h, KC_EUNSUPPORTED, "too many rows");
    k_mlp_forward<<<(unsigned)nb, 256, NP * sizeof(float), (hipStream_t)stream>>>(w_bf16, feat, rows,
                                                                                 score, act);
    return kc_check_launch(h, "k_mlp_forward");
  });
}

extern "C" kc_status kc_mlp_backward(kc_handle *h, const uint16_t *w_bf16, const float *feat,
                                     const float *act, const float *dscore, int64_t rows,
                                     float *dw, void *stream) {
  return kc_guard(h, [&]() -> kc_status {
    if (!h) return KC_EINVAL;
    KC_RETURN_IF(!w_bf16 || !feat || !act || !dscore || !dw, h, KC_EINVAL, "a pointer is NULL");
    KC_RETURN_IF(rows < 1, h, KC_EINVAL, "rows must be >= 1");
    hipStream_t st = (hipStream_t)stream;
    const int64_t chunk = 256;
    const int64_t n_chunks = (rows + chunk - 1) / chunk;
    KC_RETURN_IF(n_chunks > 65535, h, KC_EUNSUPPORTED, "too many rows for one backward call");
    const size_t gb = (size_t)rows * 3 * NH * sizeof(float);
    const size_t pb = (size_t)n_chunks * NP * sizeof(float);
    void *scr = nullptr;
    kc_status s = kc_get_scratch(h, gb + pb, &scr);
    if (s != KC_OK) return s;
    float *grad = (float *)scr;
    float *part = (float *)((char *)scr + gb);
    k_mlp_back_rows<<<(unsigned)((rows + 255) / 256), 256, NP * sizeof(float), st>>>(w_bf16, act, dscore,
                                                                                    rows, grad);
    if ((s = kc_check_launch(h, "k_mlp_back_rows")) != KC_OK) return s;
    k_mlp_back_params<<<dim3((NP + 255) / 256, (unsigned)n_chunks), 256, 0, st>>>(feat, act, grad, dscore,
                                                                                  rows, chunk, part);
    if ((s = kc_check_launch(h, "k_mlp_back_params")) != KC_OK) return s;
    k_mlp_back_sum<<<(NP + 255) / 256, 256, 0, st>>>(part, (int)n_chunks, dw);
    return kc_check_launch(h, "k_mlp_back_sum");
  });
}

extern "C" kc_status kc_mlp_loss(kc_handle *h, const float *score, const int32_t *grp_off,
                                 const int32_t *target, int32_t n_groups, int64_t rows,
                                 float *dscore, float *loss, void *stream) {
  return kc_guard(h, [&]() -> kc_status {
    if (!h) return KC_EINVAL;
    KC_RETURN_IF(!score || !grp_off || !target || !dscore || !loss, h, KC_EINVAL, "a pointer is NULL");
    KC_RETURN_IF(n_groups < 1 || rows < 1, h, KC_EINVAL, "need n_groups >= 1 and rows >= 1");
    k_mlp_loss<<<1, 256, 0, (hipStream_t)stream>>>(score, grp_off, target, n_groups, rows, dscore, loss);
    return kc_check_launch(h, "k_mlp_loss");
  });
}

extern "C" kc_status kc_mlp_adam(kc_handle *h, float *w32, uint16_t *w_bf16, const float *dw,
                                 float *m, float *v, int32_t step, float lr, void *stream) {
  return kc_guard(h, [&]() -> kc_status {
    if (!h) return KC_EINVAL;
    KC_RETURN_IF(!w32 || !w_bf16 || !dw || !m || !v, h, KC_EINVAL, "a pointer is NULL");
    KC_RETURN_IF(step < 1, h, KC_EINVAL, "step must be >= 1");
    const float c1 = (float)(1.0 - std::pow(0.9, step));
    const float c2 = (float)(1.0 - std::pow(0.999, step));
    k_mlp_adam<<<(NP + 255) / 256, 256, 0, (hipStream_t)stream>>>(w32, w_bf16, dw, m, v, c1, c2, lr);
    return kc_check_launch(h, "k_mlp_adam");
  });
}
