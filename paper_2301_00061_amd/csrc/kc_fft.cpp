// kc_fft.cpp -- farthest first traversal (Algorithm 2) from many starts at
// once: every step is one float64 objective launch over all trials, whose
// argmax per trial is that trial's next center.
#include <cmath>
#include <vector>

#include "kc_internal.h"

namespace {

struct DevMem {
  void *p = nullptr;
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
  bool alloc(size_t bytes) {
    if (hipMalloc(&p, bytes + 256) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      return false;
    }
    return true;
  }
};

}  // namespace

extern "C" kc_status kc_fft(kc_handle *h, const kc_points *pts, int32_t k, int32_t n_trials,
                            const int64_t *starts, int64_t *ids, double *obj, void *stream) {
  return kc_guard(h, [&]() -> kc_status {
    if (!h) return KC_EINVAL;
    kc_status s = kc_validate_points(h, pts);
    if (s != KC_OK) return s;
    KC_RETURN_IF(k < 1 || k > 64, h, KC_EINVAL, "k must be in [1,64] (got %d)", k);
    KC_RETURN_IF(n_trials < 1 || n_trials > 65535, h, KC_EINVAL, "n_trials must be in [1,65535]");
    KC_RETURN_IF(!starts || !ids, h, KC_EINVAL, "starts and ids are required");
    for (int t = 0; t < n_trials; ++t)
      KC_RETURN_IF(starts[t] < 0 || starts[t] >= pts->n, h, KC_EINVAL, "start %lld out of range",
                   (long long)starts[t]);
    hipStream_t st = (hipStream_t)stream;
    const int d = pts->d;
    const size_t T = (size_t)n_trials;
    DevMem d_ids, d_xy, d_obj, d_am;
    if (!d_ids.alloc(T * k * 8) || !d_xy.alloc(T * k * d * 4) || !d_obj.alloc(T * 8) ||
        !d_am.alloc(T * 8))
      return kc_fail(h, KC_ENOMEM, "fft buffers");
    // ids of the centers so far, [trial][j] compact for j centers per trial
    std::vector<int64_t> cur(T * k), next(T), step_ids;
    std::vector<double> vals(T);
    for (size_t t = 0; t < T; ++t) cur[t * k] = starts[t];
    for (int j = 1; j <= k; ++j) {
      step_ids.resize(T * j);
      for (size_t t = 0; t < T; ++t)
        for (int q = 0; q < j; ++q) step_ids[t * j + q] = cur[t * k + q];
      if (hipMemcpyAsync(d_ids.p, step_ids.data(), T * j * 8, hipMemcpyHostToDevice, st) != hipSuccess)
        return kc_fail(h, KC_EDEVICE, "fft upload");
      // coordinates [trial][j][d], the layout of kc_objective's center sets
      if ((s = kc_gather(h, pts, (const int64_t *)d_ids.p, (int)(T * j), nullptr, (float *)d_xy.p,
                         nullptr, st)))
        return s;
      if ((s = kc_objective(h, pts, n_trials, j, (const float *)d_xy.p, 64, (double *)d_obj.p,
                            (int64_t *)d_am.p, st)))
        return s;
      if (j < k) {
        if (hipMemcpyAsync(next.data(), d_am.p, T * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
          return kc_fail(h, KC_EDEVICE, "fft download");
        for (size_t t = 0; t < T; ++t) cur[t * k + j] = next[t];
      } else {
        if (hipMemcpyAsync(vals.data(), d_obj.p, T * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
          return kc_fail(h, KC_EDEVICE, "fft download");
      }
    }
    for (size_t i = 0; i < T * k; ++i) ids[i] = cur[i];
    if (obj)
      for (size_t t = 0; t < T; ++t) obj[t] = vals[t];
    return KC_OK;
  });
}
