// Per-shape autotuning of kernel variants.  The scatter (W^T) has four
// LDS-tiled forms (base, 1.5, 2 and 5 times the base number of columns per
// work-group) and two cache-direct forms, all with identical results; the
// gather (W) takes 2, 1 or 4 columns per thread (identical results); each K_UU factor has a
// circulant-FFT and a dense matrix-core form (equal up to rounding).  Which is
// faster depends on the grid size, the number of points per cell and the
// number of right-hand sides.  The tuner times each candidate with HIP events
// on the caller's stream and keeps the fastest in the plan.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "internal.h"

namespace dski {

constexpr int kScatterVariants = 7;  // 6: the grouped 3-D form (elsewhere the same kernel as 3, not timed)
constexpr int kGatherVariants = 3;
constexpr int kTuneTimes = kScatterVariants + kGatherVariants + 2 * DSKI_MAXD;

__global__ void k_fill_pm1(float* __restrict__ out, size_t len, uint64_t seed) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < len; i += (size_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    out[i] = (z >> 63) ? -0.5f : 0.5f;
  }
}

__global__ void k_fill_pm1_d(double* __restrict__ out, size_t len, uint64_t seed) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < len; i += (size_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    out[i] = (z >> 63) ? -0.5 : 0.5;
  }
}

template <class F>
static dski_status time_us(F&& fn, int reps, hipStream_t st, double* us) {
  hipEvent_t a, b;
  DSKI_HIP(hipEventCreate(&a));
  DSKI_HIP(hipEventCreate(&b));
  dski_status rc = fn();  // warm-up
  if (rc < 0) return rc;
  DSKI_HIP(hipEventRecord(a, st));
  for (int i = 0; i < reps; ++i) {
    rc = fn();
    if (rc < 0) return rc;
  }
  DSKI_HIP(hipEventRecord(b, st));
  DSKI_HIP(hipEventSynchronize(b));
  float ms = 0;
  DSKI_HIP(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *us = 1e3 * ms / reps;
  return DSKI_OK;
}

}  // namespace dski

using namespace dski;

extern "C" dski_status dski_autotune(dski_plan p, int R, double* times_host, dski_stream stream) {
  if (!p || R <= 0 || R > 32) {
    set_error("dski_autotune: bad arguments (1 <= R <= 32)");
    return DSKI_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int N = p->N;
  const int reps = 10;
  DevBuf buf;
  const size_t nv = (size_t)N * R;
  DSKI_TRY(buf.reserve(sizeof(float) * nv + 64));
  float* V = buf.as<float>();
  k_fill_pm1<<<1024, 256, 0, st>>>(V, nv, 12345);
  DSKI_HIP(hipGetLastError());
  double t[kTuneTimes] = {0};
  // scatter variants (D-SKI plans only)
  int best_s = 0;
  if (p->kind == 0) DSKI_TRY(p->grid.reserve(sizeof(double) * (size_t)p->M * R));
  double* G = p->grid.as<double>();
  // variant 6 exists in 3-D only (elsewhere it repeats variant 3): time -1, never chosen
  const int nsv = p->d == 3 ? kScatterVariants : kScatterVariants - 1;
  if (p->kind == 0 && p->d != 3) t[kScatterVariants - 1] = -1.0;
  for (int v = 0; v < (p->kind == 0 ? nsv : 0); ++v) {
    p->scatter_variant = v;
    DSKI_TRY(time_us([&]() { return scatter<float, double>(p, R, V, N, G, st); }, reps, st, &t[v]));
    if (t[v] < t[best_s]) best_s = v;
  }
  p->scatter_variant = best_s;
  // the same forms with FP64 column values (their column chunks differ, and so
  // may the fastest form); not reported, kept for the FP64 MVMs
  if (p->kind == 0) {
    DevBuf buf64;
    DSKI_TRY(buf64.reserve(sizeof(double) * nv + 64));
    double* V64 = buf64.as<double>();
    k_fill_pm1_d<<<1024, 256, 0, st>>>(V64, nv, 12345);
    DSKI_HIP(hipGetLastError());
    int best64 = 0;
    double t64[kScatterVariants] = {0};
    for (int v = 0; v < nsv; ++v) {
      p->scatter_variant64 = v;
      DSKI_TRY(time_us([&]() { return scatter<double, double>(p, R, V64, N, G, st); }, reps, st, &t64[v]));
      if (t64[v] < t64[best64]) best64 = v;
    }
    p->scatter_variant64 = best64;
    DSKI_HIP(hipStreamSynchronize(st));
    buf64.release();
    DSKI_TRY((scatter<float, double>(p, R, V, N, G, st)));  // the FP32 columns' grid for the stages below
  }
  // gather: columns per thread (on the scattered grid; writes into the second half of V)
  int best_g = 0;
  if (p->kind == 0) {
    DevBuf ybuf;
    DSKI_TRY(ybuf.reserve(sizeof(float) * nv + 64));
    float* Y = ybuf.as<float>();
    for (int v = 0; v < kGatherVariants; ++v) {
      p->gather_variant = v;
      double* tg = t + kScatterVariants;
      DSKI_TRY(time_us([&]() { return gather<float, double>(p, R, G, V, N, Y, N, 1.0, 1.0, nullptr, st); }, reps, st,
                       &tg[v]));
      if (tg[v] < tg[best_g]) best_g = v;
    }
    DSKI_HIP(hipStreamSynchronize(st));
    ybuf.release();
  }
  p->gather_variant = best_g;
  // K_UU per axis: FFT or dense matrix-core product (on the scattered grid)
  for (int a = 0; a < (p->kind == 0 ? p->d : 0); ++a) {
    int best = 0;
    for (int v = 0; v < 2; ++v) {
      double* ta = t + kScatterVariants + kGatherVariants + 2 * a;
      if (p->kernel == kKernelSpline || (v == 1 && p->ax[a].m > kDenseMaxM)) {
        // no dense form on this axis (or no separable factor at all): -1
        ta[v] = -1.0;
        continue;
      }
      DSKI_TRY(time_us([&]() { return kuu_axis<double>(p, R, G, st, -1, a, v); }, reps, st, &ta[v]));
      if (ta[v] < ta[best]) best = v;
    }
    p->kuu_variant[a] = best;
  }
  DSKI_HIP(hipStreamSynchronize(st));
  buf.release();
  if (times_host)
    for (int i = 0; i < kTuneTimes; ++i) times_host[i] = t[i];
  return DSKI_OK;
}

extern "C" dski_status dski_set_variants(dski_plan p, int scatter_variant, int gather_variant) {
  if (!p || scatter_variant < 0 || scatter_variant >= kScatterVariants || gather_variant < 0 ||
      gather_variant >= kGatherVariants) {
    set_error("dski_set_variants: bad arguments");
    return DSKI_EINVAL;
  }
  p->scatter_variant = scatter_variant;
  p->scatter_variant64 = scatter_variant;
  p->gather_variant = gather_variant;
  return DSKI_OK;
}

extern "C" dski_status dski_set_graph(dski_plan p, int on) {
  if (!p || (on != 0 && on != 1)) {
    set_error("dski_set_graph: bad arguments");
    return DSKI_EINVAL;
  }
  p->use_graph = on;
  return DSKI_OK;
}

extern "C" dski_status dski_set_kuu_variant(dski_plan p, int axis, int variant) {
  if (!p || p->kind != 0 || axis < 0 || axis >= p->d || variant < 0 || variant > 1) {
    set_error("dski_set_kuu_variant: bad arguments");
    return DSKI_EINVAL;
  }
  p->kuu_variant[axis] = variant;
  return DSKI_OK;
}

// ---------------------------------------------------------------- per-shape cache
// One text line per tuned shape:
//   dski-tune-v1 <arch> kind=<0|1> d=<d> S=<S> n=<n> m=<m0>x<m1>x<m2> R=<R> : <scatter> <scatter64> <gather> <kuu0> <kuu1> <kuu2>
// The key holds everything the timings depend on (device architecture, plan
// kind, dimension, stencil, points, grid and right-hand sides).
static std::mutex tune_cache_mu;

static std::string tune_key(dski_plan p, int R) {
  hipDeviceProp_t prop{};
  int dev = 0;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  for (char& c : arch)
    if (c == ' ' || c == ':') c = '_';
  char buf[256];
  int m[3] = {0, 0, 0};
  for (int a = 0; a < p->d && a < 3; ++a) m[a] = p->ax[a].m;
  snprintf(buf, sizeof(buf), "dski-tune-v1 %s kind=%d d=%d S=%d n=%d m=%dx%dx%d R=%d", arch.c_str(), p->kind, p->d,
           p->S, p->n, m[0], m[1], m[2], R);
  return buf;
}

extern "C" dski_status dski_autotune_cached(dski_plan p, int R, const char* cache_path, int* hit_host,
                                            double* times_host, dski_stream stream) {
  if (!p || R <= 0 || R > 32 || !cache_path || !cache_path[0]) {
    set_error("dski_autotune_cached: bad arguments (1 <= R <= 32, cache path required)");
    return DSKI_EINVAL;
  }
  const std::string key = tune_key(p, R);
  std::lock_guard<std::mutex> lock(tune_cache_mu);
  if (FILE* f = fopen(cache_path, "r")) {
    char line[512];
    bool found = false;
    int v[6] = {0, 0, 0, 0, 0, 0};
    while (fgets(line, sizeof(line), f)) {
      const char* colon = strstr(line, " : ");
      if (!colon || (size_t)(colon - line) != key.size() || strncmp(line, key.c_str(), key.size()) != 0) continue;
      int w[6];
      if (sscanf(colon + 3, "%d %d %d %d %d %d", &w[0], &w[1], &w[2], &w[3], &w[4], &w[5]) == 6 && w[0] >= 0 &&
          w[0] < kScatterVariants && w[1] >= 0 && w[1] < kScatterVariants && w[2] >= 0 && w[2] < kGatherVariants &&
          w[3] >= 0 && w[3] <= 1 && w[4] >= 0 && w[4] <= 1 && w[5] >= 0 && w[5] <= 1) {
        for (int i = 0; i < 6; ++i) v[i] = w[i];
        found = true;  // the last matching line wins
      }
    }
    fclose(f);
    if (found) {
      p->scatter_variant = v[0];
      p->scatter_variant64 = v[1];
      p->gather_variant = v[2];
      for (int a = 0; a < DSKI_MAXD; ++a) p->kuu_variant[a] = (a < p->d && p->ax[a].m <= kDenseMaxM) ? v[3 + a] : 0;
      if (hit_host) *hit_host = 1;
      if (times_host)
        for (int i = 0; i < kTuneTimes; ++i) times_host[i] = -1.0;  // not measured
      return DSKI_OK;
    }
  }
  DSKI_TRY(dski_autotune(p, R, times_host, stream));
  if (hit_host) *hit_host = 0;
  FILE* f = fopen(cache_path, "a");
  if (!f) {
    set_error("dski_autotune_cached: cannot append to %s", cache_path);
    return DSKI_EINVAL;
  }
  fprintf(f, "%s : %d %d %d %d %d %d\n", key.c_str(), p->scatter_variant, p->scatter_variant64, p->gather_variant,
          p->kuu_variant[0], p->kuu_variant[1], p->kuu_variant[2]);
  fclose(f);
  return DSKI_OK;
}
