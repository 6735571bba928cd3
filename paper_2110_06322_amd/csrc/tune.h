// Tuner helpers shared by the operator/preconditioner tuner and the batch tuner.
#pragma once

#include <hip/hip_runtime_api.h>

#include <functional>
#include <map>
#include <string>
#include <vector>

#include "schwarz.h"

namespace cpm {
namespace tune {

using Cache = std::map<std::string, std::vector<int>>;

Cache read_cache(const char* path);                  // empty when missing or unreadable
void write_cache(const char* path, const Cache& c);  // no-op for a null path
int log2i(double v);
std::string device_tag();                            // e.g. "gfx950-cu256"
// a cached subdomain-solve entry, for preconditioners with or without the packet layout
bool valid_schwarz(const std::vector<int>& v, bool packets, bool fp32, int nrhs);
// candidate kernels; all candidates for one layout compute bit-identical results
std::vector<SchwarzCfg> schwarz_candidates(bool packets, bool fp32, int nrhs);
// false when f's kernel cannot be launched at this size (its local memory
// exceeds the limit); other launch errors throw
bool launchable(const std::function<hipError_t()>& f);
// mean milliseconds of `reps` launches of f after two warm-up launches
double time_ms(const std::function<hipError_t()>& f, int reps, hipStream_t s);

}  // namespace tune
}  // namespace cpm
