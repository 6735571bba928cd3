// Coarse level of the two-level Schwarz preconditioner (see coarse.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace cpm {

// one instance's coarse space, as the kernels see it
struct DevCoarse {
  int32_t n = 0;                  // coarse unknowns (subdomains); 0 = no coarse level
  int32_t mode = 0;               // cpm_coarse: 1 additive, 2 coarse first
  int64_t nA = 0;
  const int32_t* own_ptr = nullptr;   // [n+1]: nodes owned by subdomain j are own_idx[own_ptr[j] .. own_ptr[j+1])
  const int32_t* own_idx = nullptr;   // [nA], ascending within a subdomain
  const int32_t* owner = nullptr;     // [nA]
  const double* ainv = nullptr;       // [n*n], row-major inverse of the Galerkin matrix R0 A R0^T
  int64_t vec_off = 0;            // node offset inside packed batch vectors
  int64_t coff = 0;               // offset of this instance inside packed coarse vectors
};

hipError_t coarse_restrict(const DevCoarse& C, int R, const double* r, double* c, hipStream_t s);
hipError_t coarse_solve(const DevCoarse& C, int R, const double* c, double* e, hipStream_t s);
hipError_t coarse_prolong(const DevCoarse& C, int R, const double* e, double* z, bool add, hipStream_t s);
hipError_t coarse_indicators(const DevCoarse& C, int j0, double* x, hipStream_t s);
hipError_t coarse_sub(int64_t n, const double* a, const double* b, double* y, hipStream_t s);

}  // namespace cpm
