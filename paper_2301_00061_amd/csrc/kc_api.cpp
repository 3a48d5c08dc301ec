// kc_api.cpp -- handle lifetime, error reporting, scratch memory, argument
// validation, the forward-error margins and the bound-kernel autotuner.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>

#include "kc_internal.h"

kc_status kc_fail(kc_handle *h, kc_status st, const char *fmt, ...) {
  if (h) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(h->err, sizeof(h->err), fmt, ap);
    va_end(ap);
  }
  return st;
}

kc_status kc_check_launch(kc_handle *h, const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return kc_fail(h, KC_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return KC_OK;
}

kc_status kc_get_scratch(kc_handle *h, size_t bytes, void **p) {
  if (bytes == 0) bytes = 256;
  if (bytes > h->scratch_bytes) {
    if (h->scratch) {
      // work already enqueued may still read the old buffer
      hipError_t e = hipDeviceSynchronize();
      if (e != hipSuccess) return kc_fail(h, KC_EDEVICE, "scratch grow: %s", hipGetErrorString(e));
      (void)hipFree(h->scratch);
      h->scratch = nullptr;
      h->scratch_bytes = 0;
    }
    size_t nb = bytes + bytes / 4;
    nb = (nb + 4095) & ~(size_t)4095;
    if (hipMalloc(&h->scratch, nb) != hipSuccess) {
      (void)hipGetLastError();
      h->scratch = nullptr;
      return kc_fail(h, KC_ENOMEM, "scratch allocation of %zu bytes failed", nb);
    }
    h->scratch_bytes = nb;
  }
  *p = h->scratch;
  return KC_OK;
}

// ------------------------------------------------------------- margins ---

extern "C" double kc_rel_margin(int d) {
  const double nu = (double)(d + 3) * 0x1p-24;
  return nu / (1.0 - nu);
}

extern "C" double kc_abs_margin(int d) { return (double)(d + 3) * 0x1p-126; }

float kc_round_up_f32(double v) {
  if (!(v < (double)FLT_MAX)) return INFINITY;
  float f = (float)v;
  if ((double)f < v) f = nextafterf(f, INFINITY);
  return f;
}

float kc_round_down_f32(double v) {
  if (!(v > -(double)FLT_MAX)) return -INFINITY;
  float f = (float)v;
  if ((double)f > v) f = nextafterf(f, -INFINITY);
  return f;
}

float kc_thr_gt(double T, int d) {
  if (std::isinf(T)) return T > 0 ? INFINITY : -INFINITY;
  return kc_round_up_f32(T * (1.0 + kc_rel_margin(d) + 0x1p-50) + kc_abs_margin(d));
}

float kc_thr_lt(double T, int d) {
  if (std::isinf(T)) return T > 0 ? INFINITY : -INFINITY;
  return kc_round_down_f32(T * (1.0 - kc_rel_margin(d) - 0x1p-50) - kc_abs_margin(d));
}

double kc_lower_from_f32(float v, int d) {
  double r = (double)v * (1.0 - kc_rel_margin(d) - 0x1p-50) - kc_abs_margin(d);
  return r > 0.0 ? r : 0.0;
}

double kc_upper_from_f32(float v, int d) {
  return (double)v * (1.0 + kc_rel_margin(d) + 0x1p-50) + kc_abs_margin(d);
}

// ---------------------------------------------------------- validation ---

kc_status kc_validate_points(kc_handle *h, const kc_points *p) {
  KC_RETURN_IF(!p, h, KC_EINVAL, "points struct is NULL");
  KC_RETURN_IF(!p->x, h, KC_EINVAL, "points.x is NULL");
  KC_RETURN_IF(p->d < 1 || p->d > 16, h, KC_EINVAL, "d must be in [1,16] (got %d)", p->d);
  KC_RETURN_IF(p->n < 1 || p->n >= ((int64_t)1 << 31), h, KC_EINVAL,
               "n must be in [1, 2^31) (got %lld)", (long long)p->n);
  KC_RETURN_IF(p->ld < p->n, h, KC_EINVAL, "ld (%lld) < n (%lld)", (long long)p->ld,
               (long long)p->n);
  KC_RETURN_IF(p->ld % 4 != 0, h, KC_EINVAL, "ld must be a multiple of 4 (got %lld)",
               (long long)p->ld);
  KC_RETURN_IF(((uintptr_t)p->x & 15) != 0, h, KC_EINVAL, "points.x must be 16-byte aligned");
  return KC_OK;
}

kc_status kc_validate_nodes(kc_handle *h, const kc_nodes *m, const kc_points *p) {
  (void)p;
  KC_RETURN_IF(!m, h, KC_EINVAL, "nodes struct is NULL");
  KC_RETURN_IF(m->n_nodes < 1, h, KC_EINVAL, "n_nodes must be >= 1 (got %d)", m->n_nodes);
  KC_RETURN_IF(m->n_boxes < 0, h, KC_EINVAL, "n_boxes must be >= 0");
  KC_RETURN_IF(m->k_max < 1 || m->k_max > 64, h, KC_EINVAL, "k_max must be in [1,64] (got %d)",
               m->k_max);
  KC_RETURN_IF(!m->box_off, h, KC_EINVAL, "box_off is NULL");
  KC_RETURN_IF(m->n_boxes > 0 && (!m->lo || !m->hi), h, KC_EINVAL, "lo/hi is NULL");
  return KC_OK;
}

kc_status kc_validate_refs(kc_handle *h, const kc_refs *r, const kc_nodes *m) {
  (void)m;
  if (!r) return KC_OK;
  KC_RETURN_IF(!r->ref_off, h, KC_EINVAL, "refs.ref_off is NULL");
  KC_RETURN_IF(r->n_refs < 0, h, KC_EINVAL, "refs.n_refs < 0");
  KC_RETURN_IF(r->max_per_box < 0 || r->max_per_box > 64, h, KC_EINVAL,
               "refs.max_per_box must be in [0,64]");
  KC_RETURN_IF(r->n_refs > 0 && !r->ref, h, KC_EINVAL, "refs.ref is NULL");
  return KC_OK;
}

// -------------------------------------------------------------- handle ---

extern "C" kc_status kc_create(kc_handle **out, int device, const char *tune_cache_path) {
  if (!out) return KC_EINVAL;
  *out = nullptr;
  int nd = 0;
  if (hipGetDeviceCount(&nd) != hipSuccess || nd < 1) {
    (void)hipGetLastError();
    return KC_EDEVICE;
  }
  if (device < 0 || device >= nd) return KC_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return KC_EDEVICE;
  kc_handle *h = new (std::nothrow) kc_handle();
  if (!h) return KC_ENOMEM;
  h->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    h->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    if (prop.sharedMemPerBlock > 0) h->lds_per_block = prop.sharedMemPerBlock;
    if (h->lds_per_block > 65536) h->lds_per_block = 65536;
  }
  if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess ||
      hipEventCreate(&h->ev2) != hipSuccess || hipEventCreate(&h->ev3) != hipSuccess) {
    kc_destroy(h);
    return KC_EDEVICE;
  }
  if (kc_noalloc_setup(h) != KC_OK) {
    kc_destroy(h);
    return KC_EDEVICE;
  }
  if (tune_cache_path && *tune_cache_path) {
    try {  // no C++ exception crosses the ABI
      h->tune_path = tune_cache_path;
      kc_tune_load(h);
    } catch (...) {
      kc_destroy(h);
      return KC_ENOMEM;
    }
  }
  *out = h;
  return KC_OK;
}

extern "C" void kc_destroy(kc_handle *h) {
  if (!h) return;
  if (h->scratch) {
    (void)hipDeviceSynchronize();
    (void)hipFree(h->scratch);
  }
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  if (h->ev2) (void)hipEventDestroy(h->ev2);
  if (h->ev3) (void)hipEventDestroy(h->ev3);
  delete h;
}

extern "C" const char *kc_last_error(const kc_handle *h) { return h ? h->err : "null handle"; }

// ------------------------------------------------------------ autotune ---

static int bucket_log2(int64_t v) {
  int b = 0;
  while (v > 1) {
    v >>= 1;
    ++b;
  }
  return b;
}

void kc_tune_key(char *buf, size_t size, int d, bool with_cand, int n_nodes, int k_max, int64_t n) {
  const int kb = k_max <= 4 ? 4 : k_max <= 8 ? 8 : k_max <= 16 ? 16 : 64;
  snprintf(buf, size, "d%d_c%d_nn%d_k%d_n%d", d, (int)with_cand, bucket_log2(n_nodes), kb,
           bucket_log2(n) / 2);
}

// Cache file: one line per shape bucket, "key S NG bpc [skip]".
void kc_tune_load(kc_handle *h) {
  std::ifstream f(h->tune_path);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream ls(line);
    std::string key;
    kc_tile t{};
    if (!(ls >> key >> t.S >> t.NG >> t.bpc)) continue;
    if (!(ls >> t.skip)) t.skip = 0;
    h->tune[key] = t;
  }
}

void kc_tune_log(const char *key, const kc_tile &t, double ms) {
  static const bool on = std::getenv("KC_TUNE_VERBOSE") != nullptr;
  if (on)
    std::fprintf(stderr, "[kc_tune] %s S=%d NG=%d bpc=%d skip=%d %.4f ms\n", key, t.S, t.NG, t.bpc,
                 t.skip, ms);
}

void kc_tune_save(kc_handle *h) {
  if (h->tune_path.empty()) return;
  std::ofstream f(h->tune_path, std::ios::trunc);
  for (auto &kv : h->tune)
    f << kv.first << " " << kv.second.S << " " << kv.second.NG << " " << kv.second.bpc << " "
      << kv.second.skip << "\n";
}

extern "C" kc_status kc_autotune(kc_handle *h, const kc_points *pts, const kc_nodes *nodes,
                                 int32_t with_cand, double *best_ms, void *stream) {
  return kc_guard(h, [&]() -> kc_status {
    if (!h) return KC_EINVAL;
    kc_status s = kc_validate_points(h, pts);
    if (s != KC_OK) return s;
    s = kc_validate_nodes(h, nodes, pts);
    if (s != KC_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const int nn = nodes->n_nodes, nb = nodes->n_boxes;
    float *raw = nullptr;
    double *safe = nullptr;
    int64_t *am = nullptr, *cand = nullptr;
    if (hipMalloc(&raw, nn * sizeof(float)) != hipSuccess ||
        hipMalloc(&safe, nn * sizeof(double)) != hipSuccess ||
        hipMalloc(&am, nn * sizeof(int64_t)) != hipSuccess ||
        hipMalloc(&cand, (nb > 0 ? nb : 1) * sizeof(int64_t)) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipFree(raw);
      (void)hipFree(safe);
      (void)hipFree(am);
      (void)hipFree(cand);
      return kc_fail(h, KC_ENOMEM, "autotune output buffers");
    }
    const bool wc = with_cand != 0;
    std::vector<kc_tile> vars = kc_bound_variants(pts->d, wc, nodes->k_max);
    double best = 1e30;
    kc_tile bt = kc_default_tile(h, pts->d, wc, nn, nodes->k_max, pts->n);
    char key[96];
    kc_tune_key(key, sizeof(key), pts->d, wc, nn, nodes->k_max, pts->n);
    for (const kc_tile &t : vars) {
      float ms = 0.f;
      double tbest = 1e30;
      bool ok = true;
      for (int rep = 0; rep < 4 && ok; ++rep) {
        hipEventRecord(h->ev0, st);
        s = kc_launch_bound(h, pts, 0, nn, nb, nodes->k_max, nodes->box_off, nodes->lo, nodes->hi,
                            raw, safe, am, wc ? cand : nullptr, t, st);
        hipEventRecord(h->ev1, st);
        if (s != KC_OK) {
          ok = false;
          break;
        }
        hipEventSynchronize(h->ev1);
        hipEventElapsedTime(&ms, h->ev0, h->ev1);
        if (rep > 0 && ms < tbest) tbest = ms;  // first run is a warm-up
      }
      if (ok) kc_tune_log(key, t, tbest);
      if (ok && tbest < best) {
        best = tbest;
        bt = t;
      }
    }
    (void)hipStreamSynchronize(st);
    (void)hipFree(raw);
    (void)hipFree(safe);
    (void)hipFree(am);
    (void)hipFree(cand);
    h->err[0] = 0;
    h->tune[key] = bt;
    kc_tune_save(h);
    if (best_ms) *best_ms = best;
    return best < 1e30 ? KC_OK : kc_fail(h, KC_EDEVICE, "no variant ran");
  });
}
