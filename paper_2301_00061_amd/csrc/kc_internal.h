// kc_internal.h -- host-side internals shared by the libkc translation units:
// the handle, scratch memory, error reporting, margin thresholds and the
// launch-variant tables the autotuner picks from.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <map>
#include <new>
#include <string>
#include <string_view>
#include <vector>

#include "kc.h"

// One launch shape of the bound kernel.
struct kc_tile {
  int S;         // samples per lane per tile
  int NG;        // nodes per workgroup (running maxima held in registers)
  int bpc;       // workgroups per compute unit the grid is sized for (bound
                 // kernel) / wavefronts per SIMD (tightening kernel)
  int skip = 0;  // tightening: wavefront tiles settled from their bounding box
};

struct kc_handle {
  int device = 0;
  int n_cu = 256;
  size_t lds_per_block = 65536;
  char err[512] = {0};  // message of the last failure (no allocation on error paths)
  void *scratch = nullptr;
  size_t scratch_bytes = 0;
  // device address of the static scratch array of kc_lower_bound_noalloc on
  // this handle's device (taken once per device at kc_create)
  void *noalloc_scratch = nullptr;
  std::string tune_path;
  // shape bucket -> chosen tile; transparent comparator, so a lookup by a
  // key in a stack buffer allocates nothing
  std::map<std::string, kc_tile, std::less<>> tune;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr, ev3 = nullptr;
  // flags and tile offsets of the last kc_reduce_count, for kc_reduce_compact
  struct {
    const float *x = nullptr;
    int64_t n = 0;
    void *scratch = nullptr;
    size_t keep_bytes = 0, cnt_bytes = 0, off_bytes = 0, bsum_bytes = 0;
  } red;
};

kc_status kc_fail(kc_handle *h, kc_status st, const char *fmt, ...);
// Returns at least `bytes` of device scratch owned by the handle. Growing the
// buffer synchronises the device first (work in flight may still use it).
kc_status kc_get_scratch(kc_handle *h, size_t bytes, void **p);
// Maps hipGetLastError after a launch to KC_EDEVICE.
kc_status kc_check_launch(kc_handle *h, const char *what);

// Margin thresholds (float32 values compared against float32 distances).
// For a float32 squared distance v_hat of exact value v:
//   v_hat > thr_gt(T)   implies v > T,
//   v_hat < thr_lt(T)   implies v < T,
//   v <= T              implies v_hat <= thr_gt(T).
float kc_thr_gt(double T, int d);
float kc_thr_lt(double T, int d);
// float32 nearest to v in the stated direction.
float kc_round_up_f32(double v);
float kc_round_down_f32(double v);
// Rigorous float64 bounds from a float32 value: lower (never negative) / upper.
double kc_lower_from_f32(float v, int d);
double kc_upper_from_f32(float v, int d);

kc_status kc_validate_points(kc_handle *h, const kc_points *p);
kc_status kc_validate_nodes(kc_handle *h, const kc_nodes *m, const kc_points *p);
kc_status kc_validate_refs(kc_handle *h, const kc_refs *r, const kc_nodes *m);

// Bound-kernel launch (implemented in kc_bound.hip); `t` selects the variant.
// mode 0: lower bound (optionally with candidates), mode 1: float32 objective.
// fixed_scratch (nullable): device memory of fixed_bytes for the per-split
// partial keys instead of the handle's scratch; a launch that needs more
// fails with KC_EINVAL and allocates nothing. cut (mode 1 only; +inf = off):
// a set whose float32 objective exceeds cut may stop early and report the
// value of some sample above the cut (a lower bound of its objective); sets
// at or below the cut get their exact value. floor (mode 1, nullable,
// device [n_nodes]): a lower bound of each set's exact objective, which lets
// the tile decisions skip tiles below it from the start (results unchanged).
kc_status kc_launch_bound(kc_handle *h, const kc_points *pts, int mode, int n_nodes,
                          int n_boxes, int k_max, const int32_t *box_off, const float *lo,
                          const float *hi, float *val_raw, double *val_bound, int64_t *argmax,
                          int64_t *cand, const kc_tile &t, hipStream_t st,
                          void *fixed_scratch = nullptr, size_t fixed_bytes = 0,
                          float cut = INFINITY, const double *floor = nullptr,
                          const float *wit_x = nullptr, const int64_t *wit_id = nullptr);
// kc_objective_screen with a witness sample per set (device: coordinates
// [n_sets][d] and the sample's index in pts, negative = none): a set whose
// float32 value at its witness exceeds cut is settled at that value before
// any tile is read. Arguments are not validated (the solver's own calls).
kc_status kc_objective_screen_witness(kc_handle *h, const kc_points *pts, int n_sets, int k,
                                      const float *centers, float cut, const double *floor,
                                      const float *wit_x, const int64_t *wit_id, double *obj,
                                      int64_t *argmax, hipStream_t st);
// Takes the device address of kc_lower_bound_noalloc's static scratch array
// for the current device (kc_bound.hip); called by kc_create with h->device
// current.
kc_status kc_noalloc_setup(kc_handle *h);
// Variants compiled for this (d, with_cand) pair.
std::vector<kc_tile> kc_bound_variants(int d, bool with_cand, int k_max);
kc_tile kc_default_tile(kc_handle *h, int d, bool with_cand, int n_nodes, int k_max, int64_t n);
// Writes the autotune table key of a shape into buf (no allocation).
void kc_tune_key(char *buf, size_t size, int d, bool with_cand, int n_nodes, int k_max, int64_t n);
void kc_tune_load(kc_handle *h);
void kc_tune_save(kc_handle *h);
// Prints one autotune measurement to stderr when KC_TUNE_VERBOSE is set.
void kc_tune_log(const char *key, const kc_tile &t, double ms);

// Tile of a tightening launch (kc_tighten.hip): the autotuner's choice for the
// shape bucket (*tuned = true), else the default; kc_tile.bpc holds the
// occupancy (wavefronts per SIMD, 0 = the compiler's choice).
kc_tile kc_tighten_tile(kc_handle *h, const kc_points *pts, const kc_nodes *nodes,
                        const kc_refs *refs, bool *tuned);
// Whether the bound kernel's table holds a tile for this shape bucket.
bool kc_bound_tuned(kc_handle *h, const kc_points *pts, const kc_nodes *nodes, bool cand);
// Tile of the float32 objective (kc_objective precision 32) for n_sets sets of
// k centers, and its sweep (kc_bound.hip; synchronous, allocates its outputs).
kc_tile kc_objective_tile(kc_handle *h, const kc_points *pts, int n_sets, int k, bool *tuned);
kc_status kc_autotune_objective(kc_handle *h, const kc_points *pts, int n_sets, int k,
                                const float *centers, hipStream_t st);

// Device gather of sample coordinates (kc_util.hip).
kc_status kc_gather(kc_handle *h, const kc_points *p, const int64_t *ids, int count,
                    const uint32_t *idx_map, float *out, int64_t *orig, hipStream_t st);

// Sample reduction in two phases (kc_reduce.hip; kc_reduce runs both):
// kc_reduce_count writes the redundancy flags and tile offsets to the handle's
// scratch and the number kept to *n_out (device); kc_reduce_compact then
// scatters the kept samples of the same points (n_keep = that number, read
// back by the caller) into x_out / idx_out, ld_out >= n_keep. No other call
// on the handle may come between them.
kc_status kc_reduce_count(kc_handle *h, const kc_points *in, const kc_nodes *open,
                          const kc_refs *refs, double beta, double alpha, int64_t *n_out,
                          hipStream_t st);
kc_status kc_reduce_compact(kc_handle *h, const kc_points *in, const uint32_t *idx_in,
                            int64_t n_keep, float *x_out, uint32_t *idx_out, int64_t ld_out,
                            hipStream_t st);

// Reorders the samples along a Morton curve over the box [lo, hi] (kc_order.hip):
// x_out / ids_out (leading dimension ld_out) receive the samples of `in` in the
// new order and their original ids (ids_in maps `in` to original ids, null:
// identity). Synchronous on `st`.
kc_status kc_spatial_order(kc_handle *h, const kc_points *in, const uint32_t *ids_in,
                           const float *lo, const float *hi, float *x_out, uint32_t *ids_out,
                           int64_t ld_out, hipStream_t st);

// Every C entry point runs its body through kc_guard, so that no C++
// exception crosses the ABI: host allocation failures become KC_ENOMEM, any
// other exception KC_EDEVICE (kc_fail itself never throws).
template <class F>
kc_status kc_guard(kc_handle *h, F &&body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc &) {
    return kc_fail(h, KC_ENOMEM, "host memory allocation failed");
  } catch (...) {
    return kc_fail(h, KC_EDEVICE, "internal error");
  }
}

#define KC_RETURN_IF(cond, h, st, ...)          \
  do {                                          \
    if (cond) return kc_fail(h, st, __VA_ARGS__); \
  } while (0)
