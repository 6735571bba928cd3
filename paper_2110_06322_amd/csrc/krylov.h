// Batched FGMRES: device state and vector-kernel launchers.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace cpm {

constexpr int kMaxRestart = 64;
constexpr int kMaxSystems = 1024;
constexpr int64_t kChunkNodes = 512;

// a contiguous node range of one instance inside the packed vectors
struct Chunk {
  int32_t inst;
  int32_t pad;
  int64_t node0;   // first node (packed numbering)
  int64_t nodes;
};

// per-system solver state in device memory (ns systems, restart m)
struct GmresState {
  int32_t m;
  int32_t pad;
  double* H;        // [ns][(m+1) x m] column-major
  double* g;        // [ns][m+1]
  double* cs;       // [ns][m]
  double* sn;       // [ns][m]
  double* y;        // [ns][m]
  double* hcol;     // [ns][m+1]  current Arnoldi column (both CGS passes summed)
  double* hv;       // [ns][m+1]  coefficients of the current update
  double* nrm2;     // [ns]
  double* beta;     // [ns]
  double* scale;    // [ns]
  double* tol_in;   // [ns]
  double* est;      // [ns]
  int32_t* act;     // [ns]
  int32_t* steps;   // [ns]
  int32_t* bad;     // [ns]
  int32_t* budget;  // [ns]  Arnoldi steps this system may still take (max_it cap)
  int32_t* n_active;
};

hipError_t vec_dots(int R, const double* V0, int64_t vstride, int m, const double* w, const Chunk* chunks,
                    int nchunks, const int32_t* act, double* part, hipStream_t s);
hipError_t vec_reduce(int R, const double* part, int m, int nchunks, const int32_t* cbeg, int ns, double* out,
                      int ld, double* accum, int accum_ld, hipStream_t s);
hipError_t vec_update(int R, const double* V0, int64_t vstride, int m, double* w, const Chunk* chunks, int nchunks,
                      const int32_t* act, const double* hv, int ld, double* part_norm, hipStream_t s);
hipError_t vec_scale(int R, const double* x, double* out, const Chunk* chunks, int nchunks, const int32_t* act,
                     const double* a, hipStream_t s);
hipError_t vec_copy(int R, const double* x, double* out, const Chunk* chunks, int nchunks, const int32_t* copy_inst,
                    hipStream_t s);
hipError_t vec_residual(int R, const double* f, const double* t, double* r, const Chunk* chunks, int nchunks,
                        double* part, hipStream_t s);
hipError_t vec_xupdate(int R, double* x, const double* Z0, int64_t zstride, const Chunk* chunks, int nchunks,
                       const int32_t* steps, const double* y, int ld, hipStream_t s);
hipError_t gmres_givens(const GmresState& S, int j, int ns, hipStream_t s);
hipError_t gmres_hsolve(const GmresState& S, int ns, hipStream_t s);
hipError_t gmres_cycle_init(const GmresState& S, int ns, hipStream_t s);

}  // namespace cpm
