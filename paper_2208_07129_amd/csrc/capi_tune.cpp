// Launch-shape tuning of the fused apply (mf_tune) and of batches
// (mf_batch_tune), with a JSON cache on disk keyed by device architecture,
// degree, quadrature, cells, columns and precision.
//
// The candidate shapes (column tile per workgroup, columns per thread,
// threads, one-shot or persistent grid) play the part of the paper's sweep of
// its GPU kernel's batch size and thread-block shape (Sec. 4, GPU benchmarks,
// tbl:batchsizeStudy): each is timed on the device and the fastest kept.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>

#include "mf_internal.h"
#include "sf_common.h"

namespace mf {

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "unknown";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

namespace {

const char* prec_name(int prec) {
  return prec == MF_FP64 ? "fp64" : prec == MF_FP32 ? "fp32" : "bf16";
}

// The cache file: one flat JSON object whose values are objects without
// nested strings.  Unreadable or malformed files read as empty.
std::map<std::string, std::string> cache_read(const char* path) {
  std::map<std::string, std::string> out;
  std::ifstream f(path);
  if (!f) return out;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string t = ss.str();
  size_t i = t.find('{');
  if (i == std::string::npos) return out;
  ++i;
  while (true) {
    const size_t k0 = t.find('"', i);
    if (k0 == std::string::npos) break;
    const size_t k1 = t.find('"', k0 + 1);
    if (k1 == std::string::npos) return {};
    const size_t colon = t.find(':', k1);
    const size_t v0 = t.find('{', k1);
    if (colon == std::string::npos || v0 == std::string::npos || v0 < colon) return {};
    int depth = 0;
    size_t v1 = v0;
    for (; v1 < t.size(); ++v1) {
      if (t[v1] == '{') ++depth;
      if (t[v1] == '}' && --depth == 0) break;
    }
    if (v1 >= t.size()) return {};
    out[t.substr(k0 + 1, k1 - k0 - 1)] = t.substr(v0, v1 - v0 + 1);
    i = v1 + 1;
  }
  return out;
}

std::string arch_prefix() { return device_arch() + "/"; }

double median(std::vector<double> v) {
  std::sort(v.begin(), v.end());
  return v.empty() ? -1.0 : v[v.size() / 2];
}

// Median time in ms of `reps` calls of fn() after `warmup`, each bracketed by
// events on s.  Returns a negative value (and the status in *st) on failure.
template <class Fn>
double time_calls(Fn fn, hipStream_t s, hipEvent_t e0, hipEvent_t e1, int warmup, int reps,
                  int* st) {
  for (int i = 0; i < warmup; ++i)
    if ((*st = fn())) return -1.0;
  std::vector<double> t;
  for (int i = 0; i < reps; ++i) {
    hipError_t err = hipEventRecord(e0, s);
    if (err != hipSuccess) {
      *st = hip_fail(err, "hipEventRecord");
      return -1.0;
    }
    if ((*st = fn())) return -1.0;
    err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err != hipSuccess) {
      *st = hip_fail(err, "hipEvent timing");
      return -1.0;
    }
    t.push_back(ms);
  }
  return median(t);
}

struct Scratch {  // device buffers and stream of one tuning run
  double* X = nullptr;
  double* Y = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~Scratch() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (X) (void)hipFree(X);
    if (Y) (void)hipFree(Y);
  }
};

}  // namespace

int cache_lookup(const char* path, const std::string& key) {
  if (!path) return -1;
  const auto db = cache_read(path);
  const auto it = db.find(key);
  if (it == db.end()) return -1;
  const size_t c = it->second.find("\"cfg\"");
  if (c == std::string::npos) return -1;
  const size_t colon = it->second.find(':', c);
  if (colon == std::string::npos) return -1;
  return (int)std::strtol(it->second.c_str() + colon + 1, nullptr, 10);
}

int cache_store(const char* path, const std::string& key, int cfg, const std::vector<double>& ms) {
  if (!path) return MF_OK;
  auto db = cache_read(path);
  std::ostringstream v;
  v << "{\"cfg\": " << cfg << ", \"ms\": [";
  for (size_t i = 0; i < ms.size(); ++i) {
    char buf[32];
    std::snprintf(buf, sizeof(buf), "%.6g", ms[i]);
    v << (i ? ", " : "") << buf;
  }
  v << "]}";
  db[key] = v.str();
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return fail(MF_ERR_ARG, std::string("cannot write the tune cache ") + tmp);
    f << "{\n";
    size_t n = 0;
    for (const auto& kv : db) f << " \"" << kv.first << "\": " << kv.second << (++n < db.size() ? ",\n" : "\n");
    f << "}\n";
    if (!f) return fail(MF_ERR_ARG, std::string("cannot write the tune cache ") + tmp);
  }
  if (std::rename(tmp.c_str(), path) != 0)
    return fail(MF_ERR_ARG, std::string("cannot replace the tune cache ") + path);
  return MF_OK;
}

}  // namespace mf

using namespace mf;

extern "C" {

int mf_tune(mf_operator* handle, int nvec, int prec, const char* cache_path) {
  if (!handle) return fail(MF_ERR_ARG, "operator is NULL");
  if (nvec < 1) return fail(MF_ERR_ARG, "nvec must be >= 1");
  if (prec != MF_FP64 && prec != MF_FP32 && prec != MF_BF16)
    return fail(MF_ERR_UNSUPPORTED, "unknown precision");
  Operator* op = reinterpret_cast<Operator*>(handle);
  const bool mixed = prec != MF_FP64;
  if (mixed && !op->box && !(op->map_box && prec == MF_FP32))
    return fail(MF_ERR_UNSUPPORTED,
                "mixed precision is built for axis-aligned cells only (FP32 on refined meshes)");
  // candidate shapes; the general-geometry and refined-map kernels have one
  // shape each, so there is nothing to choose
  std::vector<int> cand;
  if (!mixed && op->box) {
    for (int c = 0; c < kBoxCfgs; ++c)
      if (apply_box_supported(op->p, op->q, c)) cand.push_back(c);
  } else if (mixed && op->box) {
    const int n = prec == MF_FP32 ? kMixedCfgs : kMixedMfmaCfgs;
    for (int c = 0; c < n; ++c)
      if (apply_mixed_supported(op->p, op->q, c)) cand.push_back(c);
  }
  if (cand.size() < 2) return MF_OK;
  char kb[160];
  std::snprintf(kb, sizeof(kb), "p%dq%d/cells%lld/nvec%d/%s", op->p, op->q, (long long)op->ncells,
                nvec, prec_name(prec));
  const std::string key = arch_prefix() + kb;
  int& override_cfg = mixed ? op->mcfg : op->cfg;
  override_cfg = -1;  // the tuned choice applies from now on
  const int cached = cache_lookup(cache_path, key);
  if (cached >= 0 && std::find(cand.begin(), cand.end(), cached) != cand.end()) {
    op->tuned[{prec, nvec}] = cached;
    op->tuned_ms[{prec, nvec}] = std::vector<double>(mixed ? kMixedCfgs : kBoxCfgs, -1.0);
    return MF_OK;
  }
  Scratch sc;
  const size_t bytes = (size_t)op->ndofs * nvec * sizeof(double);
  hipError_t err = hipMalloc(&sc.X, bytes);
  if (err == hipSuccess) err = hipMalloc(&sc.Y, bytes);
  if (err != hipSuccess)
    return err == hipErrorOutOfMemory ? fail(MF_ERR_OOM, "hipMalloc (tuner buffers)")
                                      : hip_fail(err, "hipMalloc");
  err = hipStreamCreateWithFlags(&sc.s, hipStreamNonBlocking);
  if (err == hipSuccess) err = hipEventCreate(&sc.e0);
  if (err == hipSuccess) err = hipEventCreate(&sc.e1);
  if (err == hipSuccess) err = launch_fill_pattern(sc.X, (int64_t)op->ndofs * nvec, sc.s);
  if (err != hipSuccess) return hip_fail(err, "tuner setup");
  std::vector<double> ms(mixed ? kMixedCfgs : kBoxCfgs, -1.0);
  int best = -1;
  // two rounds over the candidates, each keeping its lower median: the first
  // candidate timed in a round otherwise pays for the device's clock ramp
  for (int round = 0; round < 2; ++round)
    for (int c : cand) {
      override_cfg = c;
      int st = MF_OK;
      const double t = time_calls(
          [&]() { return apply_dispatch(handle, sc.X, sc.Y, nvec, nvec, nvec, prec, sc.s, false); },
          sc.s, sc.e0, sc.e1, 2, 7, &st);
      if (st) {
        override_cfg = -1;
        return st;
      }
      if (ms[c] < 0.0 || t < ms[c]) ms[c] = t;
    }
  for (int c : cand)
    if (best < 0 || ms[c] < ms[best]) best = c;
  override_cfg = -1;
  op->tuned[{prec, nvec}] = best;
  op->tuned_ms[{prec, nvec}] = ms;
  return cache_store(cache_path, key, best, ms);
}

int mf_tune_info(const mf_operator* handle, int nvec, int prec, int* cfg, double* ms, int nms) {
  if (!handle) return fail(MF_ERR_ARG, "operator is NULL");
  const Operator* op = reinterpret_cast<const Operator*>(handle);
  const auto it = op->tuned.find({prec, nvec});
  if (cfg) *cfg = it == op->tuned.end() ? -1 : it->second;
  if (ms && nms > 0) {
    for (int i = 0; i < nms; ++i) ms[i] = -1.0;
    const auto jt = op->tuned_ms.find({prec, nvec});
    if (jt != op->tuned_ms.end())
      for (int i = 0; i < nms && i < (int)jt->second.size(); ++i) ms[i] = jt->second[i];
  }
  return MF_OK;
}

}  // extern "C"
