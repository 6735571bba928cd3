// Autotuner: times the candidate kernel configurations of an operator's
// one-RHS apply and of a preconditioner's subdomain solves on scratch vectors,
// keeps the fastest, and caches the choice per shape class in a JSON file
// (an object mapping class keys to integer arrays), so later operators of the
// same class skip the timing.
#include <cctype>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "common.h"
#include "schwarz.h"
#include "tune.h"

using namespace cpm;

namespace cpm {
hipError_t precond_apply_raw(const cpm_precond_s* pc, const double* r, double* z, int nrhs, hipStream_t s);
int precond_take_error(const cpm_precond_s* pc);

namespace tune {

// parse {"key": [i, j, ...], ...}; anything else yields an empty cache
Cache read_cache(const char* path) {
  Cache c;
  if (!path) return c;
  std::ifstream f(path);
  if (!f) return c;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t i = 0;
  auto skip = [&] { while (i < s.size() && std::isspace((unsigned char)s[i])) ++i; };
  skip();
  if (i >= s.size() || s[i] != '{') return Cache{};
  ++i;
  for (;;) {
    skip();
    if (i < s.size() && s[i] == '}') break;
    if (i >= s.size() || s[i] != '"') return Cache{};
    const size_t e = s.find('"', i + 1);
    if (e == std::string::npos) return Cache{};
    std::string key = s.substr(i + 1, e - i - 1);
    i = e + 1;
    skip();
    if (i >= s.size() || s[i] != ':') return Cache{};
    ++i;
    skip();
    if (i >= s.size() || s[i] != '[') return Cache{};
    ++i;
    std::vector<int> v;
    for (;;) {
      skip();
      if (i < s.size() && s[i] == ']') { ++i; break; }
      char* end = nullptr;
      long x = std::strtol(s.c_str() + i, &end, 10);
      if (end == s.c_str() + i) return Cache{};
      v.push_back((int)x);
      i = (size_t)(end - s.c_str());
      skip();
      if (i < s.size() && s[i] == ',') ++i;
    }
    c[key] = v;
    skip();
    if (i < s.size() && s[i] == ',') { ++i; continue; }
    skip();
    if (i < s.size() && s[i] == '}') break;
    return Cache{};
  }
  return c;
}

void write_cache(const char* path, const Cache& c) {
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) return;
    f << "{\n";
    size_t n = 0;
    for (const auto& kv : c) {
      f << "  \"" << kv.first << "\": [";
      for (size_t j = 0; j < kv.second.size(); ++j) f << (j ? ", " : "") << kv.second[j];
      f << "]" << (++n < c.size() ? "," : "") << "\n";
    }
    f << "}\n";
  }
  std::rename(tmp.c_str(), path);
}

int log2i(double v) { return v <= 1 ? 0 : (int)std::lround(std::log2(v)); }

bool valid_schwarz(const std::vector<int>& v, bool packets, bool fp32, int nrhs) {
  if (v.size() != 3) return false;
  const bool variant_ok = packets ? (v[0] == kSchwarzPacket || v[0] == kSchwarzPacketFlags ||
                                     (v[0] == kSchwarzPacketLevel && nrhs == 1))
                                  : (v[0] == kSchwarzFlags || v[0] == kSchwarzValueFlags);
  return variant_ok && v[1] >= 64 && v[1] <= (packets ? packet_max_threads(fp32, nrhs, v[0] == kSchwarzPacketFlags) : 1024) && v[1] % 64 == 0 &&
         (v[2] == 0 || v[2] == 1);
}

// The packet kernels sum a row in another order than the two one-row-per-
// wavefront kernels, so only they are candidates for a packet layout.
std::vector<SchwarzCfg> schwarz_candidates(bool packets, bool fp32, int nrhs) {
  std::vector<SchwarzCfg> out;
  std::vector<int> variants = packets ? std::vector<int>{kSchwarzPacket, kSchwarzPacketFlags}
                                      : std::vector<int>{kSchwarzFlags, kSchwarzValueFlags};
  if (packets && nrhs == 1) variants.push_back(kSchwarzPacketLevel);   // level waits: one right-hand side
  for (int variant : variants)
    for (int threads : {256, 512, 768, 1024})
      for (int sleep : {0, 1}) {
        if (variant == kSchwarzFlags && sleep == 0) continue;   // the flag kernel always backs off
        if (packets ? threads > packet_max_threads(fp32, nrhs, variant == kSchwarzPacketFlags) : threads == 768)
          continue;
        SchwarzCfg c;
        c.variant = variant;
        c.threads = threads;
        c.sleep = sleep;
        out.push_back(c);
      }
  return out;
}

std::string device_tag() {
  int dev = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string name = prop.gcnArchName;
  const size_t colon = name.find(':');
  if (colon != std::string::npos) name = name.substr(0, colon);
  return name + "-cu" + std::to_string(prop.multiProcessorCount);
}

bool launchable(const std::function<hipError_t()>& f) {
  const hipError_t e = f();
  if (e == hipErrorInvalidConfiguration) return false;   // rejected before any launch
  hip_check(e, "tune launch");
  return true;
}

double time_ms(const std::function<hipError_t()>& f, int reps, hipStream_t s) {
  hipEvent_t a, b;
  hip_check(hipEventCreate(&a), "tune");
  hip_check(hipEventCreate(&b), "tune");
  hip_check(f(), "tune warm-up");
  hip_check(f(), "tune warm-up");
  hip_check(hipEventRecord(a, s), "tune");
  for (int i = 0; i < reps; ++i) hip_check(f(), "tune launch");
  hip_check(hipEventRecord(b, s), "tune");
  hip_check(hipEventSynchronize(b), "tune");
  float ms = 0;
  hip_check(hipEventElapsedTime(&ms, a, b), "tune");
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms / reps;
}

}  // namespace tune
}  // namespace cpm

using namespace cpm::tune;

cpm_status cpm_autotune(cpm_operator* op, cpm_precond* pc, int32_t nrhs, const char* cache_path, int32_t force,
                        void* stream, cpm_tune_result* out) {
  try {
    if (!op || !out) fail(CPM_ERR_ARG, "null argument");
    if (pc && pc->op != op) fail(CPM_ERR_ARG, "preconditioner built for another operator");
    if (nrhs != 1 && nrhs != 2 && nrhs != 4) fail(CPM_ERR_ARG, "nrhs must be 1, 2 or 4");
    std::memset(out, 0, sizeof(*out));
    hipStream_t s = (hipStream_t)stream;
    const int reps = 10;
    Cache cache = read_cache(cache_path);
    bool dirty = false, all_cached = true;
    const std::string dev = device_tag();
    const int64_t n = op->band->nA;
    DevBuf<double> x, y;
    x.alloc((size_t)std::max<int64_t>(n, 1) * nrhs);
    y.alloc((size_t)std::max<int64_t>(n, 1) * nrhs);
    // x = 1.0000002 everywhere (hi and lo words 0x3ff00000): finite, non-trivial values
    hip_check(hipMemsetD32Async((hipDeviceptr_t)x.p, 0x3ff00000, (size_t)n * nrhs * 2, s), "tune fill");

    // ---- operator apply (the kernel choice exists for one right-hand side)
    {
      char key[160];
      std::snprintf(key, sizeof key, "apply|%s|d%dp%dr%d|nA2^%d", dev.c_str(), op->I.d, op->I.p, nrhs,
                    log2i((double)n));
      std::vector<int> cand = {kApplyPerTile};
      if (nrhs == 1) {
        cand = {kApplyPipelined, kApplyPerTile};
        if (op->twopass) cand.push_back(kApplyTwoPass);
      }
      auto it = cache.find(key);
      if (!force && it != cache.end() && !it->second.empty() &&
          (it->second[0] == kApplyPipelined || it->second[0] == kApplyPerTile ||
           (it->second[0] == kApplyTwoPass && op->twopass && nrhs == 1))) {
        op->apply_variant = it->second[0];
      } else {
        all_cached = false;
        double best = 1e30;
        int bestv = kApplyPipelined;
        for (const int v : cand) {
          const double ms = time_ms([&] { return launch_apply(op->apply_args(), nrhs, v, x.p, y.p, s); }, reps, s);
          if (ms < best) { best = ms; bestv = v; }
        }
        op->apply_variant = bestv;
        cache[key] = {bestv};
        dirty = true;
      }
      out->apply_variant = op->apply_variant;
      auto f = [&] { return launch_apply(op->apply_args(), nrhs, op->apply_variant, x.p, y.p, s); };
      out->apply_ms = time_ms(f, reps, s);
    }

    // ---- subdomain solves
    if (pc) {
      char key[200];
      std::snprintf(key, sizeof key, "schwarz|%s|%s%s|r%d|rows2^%d|levels2^%d|parts2^%d", dev.c_str(),
                    pc->P.fp32 ? "fp32" : "fp64", pc->packets ? "|packets" : "", nrhs, log2i((double)pc->max_rows), log2i((double)pc->max_levels),
                    log2i((double)pc->host.nparts));
      auto it = cache.find(key);
      if (!force && it != cache.end() && valid_schwarz(it->second, pc->packets, pc->P.fp32 != 0, nrhs)) {
        pc->cfg.variant = it->second[0];
        pc->cfg.threads = it->second[1];
        pc->cfg.sleep = it->second[2];
      } else {
        all_cached = false;
        double best = 1e30;
        SchwarzCfg bestc = pc->cfg;
        for (const SchwarzCfg& c : schwarz_candidates(pc->packets, pc->P.fp32 != 0, nrhs)) {
          pc->cfg = c;
          auto run = [&] { return precond_apply_raw(pc, x.p, y.p, nrhs, s); };
          if (!launchable(run)) continue;
          const double ms = time_ms(run, reps, s);
          if (ms < best) { best = ms; bestc = c; }
        }
        if (best >= 1e30) {
          pc->cfg = bestc;
          fail(CPM_ERR_ARG, "subdomains too large for the local-memory budget at this nrhs/precision");
        }
        pc->cfg = bestc;
        cache[key] = {bestc.variant, bestc.threads, bestc.sleep};
        dirty = true;
      }
      if (precond_take_error(pc)) fail(CPM_ERR_DEVICE, "a subdomain solve timed out while tuning");
      out->schwarz_variant = pc->cfg.variant;
      out->schwarz_threads = pc->cfg.threads;
      out->schwarz_sleep = pc->cfg.sleep;
      out->precond_ms = time_ms([&] { return precond_apply_raw(pc, x.p, y.p, nrhs, s); }, reps, s);
    }
    hip_check(hipStreamSynchronize(s), "tune");
    // cached single-solve workspaces were built with the old choices
    op->solve_cache.reset();
    op->solve_cache_key = -1;
    out->from_cache = all_cached ? 1 : 0;
    if (dirty) write_cache(cache_path, cache);
    return CPM_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed in cpm_autotune");
    return CPM_ERR_OOM;
  }
}
