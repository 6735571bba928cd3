// Schwarz preconditioner: host setup result and the device-side view.
#pragma once

#include <cstdint>
#include <vector>

#include "coarse.h"
#include "common.h"

namespace cpm {

struct SchwarzHost {
  struct Sub {
    int n = 0;
    int64_t nnz = 0;
    int levels = 0;
    std::vector<int32_t> rows;     // global active indices of Omega_j, local order
    std::vector<int32_t> perm;     // input slot q takes local row perm[q] (key order)
    std::vector<int32_t> operm;    // solution slot q is local row operm[q]
    std::vector<uint16_t> schedL, schedU;  // level-ordered rows of the forward / backward sweeps
    std::vector<int32_t> levL, levU;       // level of the row at each schedule position
    std::vector<int64_t> lptr, uptr;
    std::vector<uint16_t> lcol, ucol;
    std::vector<double> lval, uval, dinv;
  };
  int nparts = 0;
  int64_t global_nnz = 0;
  std::vector<int32_t> owner;
  std::vector<Sub> subs;
};

void build_schwarz_host(const cpm_band_s& B, double c, const cpm_precond_opts& o, SchwarzHost& S);
void extension_row(const cpm_band_s& B, int64_t n, std::vector<int32_t>& cols, std::vector<double>& w);
void operator_row(const cpm_band_s& B, double c, int64_t i, std::vector<int32_t>& cols, std::vector<double>& vals,
                  std::vector<int32_t>& scratch_c, std::vector<double>& scratch_w);

// One subdomain as the kernel sees it (offsets into the preconditioner's packed arrays).
struct DevSub {
  int64_t row_off;   // into in_idx / out_idx / dinv / recL / recU (n entries)
  int64_t lbase;     // first stored entry of the subdomain in lcol / lval
  int64_t ubase;     // first stored entry in ucol / uval
  int64_t pk_off;    // first packet of the forward sweep in pk (backward packets follow)
  int32_t n;
  int32_t npkL;      // packets of the forward / backward sweeps (packet layout only)
  int32_t npkU;
  int32_t pad;
};

// One row of a triangular sweep, in schedule order: local row (bits 48..63),
// stored entries (bits 32..47), offset of its first entry from the subdomain's
// entry base (bits 0..31). Entries are stored in schedule order.
struct DevPC {
  int32_t nparts;
  int32_t fp32;                 // values (lval, uval, dinv) are float
  const DevSub* subs;
  const int32_t* in_idx;        // global node feeding input slot q
  const int32_t* out_idx;       // global node of solution slot q, bit 31 set when owned
  const int32_t* gL;            // global node of the row at each forward-sweep position
  const uint64_t* recL;         // per subdomain (at row_off): forward sweep records
  const uint64_t* recU;         //   backward sweep records
  const uint32_t* pk;           // packets of same-level schedule positions (packet layout), else null
  const uint16_t* lcol;
  const uint16_t* ucol;
  const void* lval;
  const void* uval;
  const void* dinv;
  int32_t* error_flag;          // set when a bounded wait expires
  int64_t vec_off;              // node offset of this instance inside packed batch vectors
};

int64_t next_serial();

// kernel configuration of the subdomain solves (chosen by the tuner)
constexpr int kSchwarzFlags = 0;        // LDS value array plus per-row completion flags
constexpr int kSchwarzValueFlags = 1;   // values double as flags (forward and backward arrays)
constexpr int kSchwarzPacket = 2;       // values as flags, up to four same-level rows per wavefront
constexpr int kSchwarzPacketFlags = 3;  // packets with per-row completion flags (less local memory)
// packets, values in two LDS arrays, one right-hand side; a packet waits until the
// sweep's count of completed rows reaches the first position of its level (levels
// then start one after another, so the count certifies every lower level)
constexpr int kSchwarzPacketLevel = 4;
// Packet layout: consecutive schedule positions of one level and one length
// class are grouped into packets of at most kPacketRows rows; a packet word
// holds its first position (bits 4..19), its class (bits 2..3), its row count
// minus one (bits 0..1) and how far its first position lies past the first
// position of its level (bits 20..31, at most 4095: a wider level makes later
// packets wait for some rows of their own level, which is slower, not wrong). Each row is solved by kPacketLanes lanes, each
// taking at most packet_slots(class) of its entries (kPacketEntries at most).
constexpr int kPacketRows = 4;
constexpr int kPacketLanes = 16;
constexpr int kPacketEntries = 12;
// length class of a factor row: entry slots per lane 4, 8 or 12
inline int packet_class(int64_t len) { return len <= 4 * kPacketLanes ? 0 : len <= 8 * kPacketLanes ? 1 : 2; }
constexpr int packet_slots(int cls) { return 4 * (cls + 1); }
// threads of a packet workgroup at most: 768 (48 rows in flight, up to 170
// registers per lane) where the kernel fits that register budget (FP32 factors
// with 1 or 2 right-hand sides; the completion-flag form with one FP64
// right-hand side), else 512 (up to 256 registers)
constexpr int packet_max_threads(bool fp32, int nrhs, bool flags) {
  return (fp32 && nrhs <= 2) || (nrhs == 1 && flags) ? 768 : 512;
}
constexpr size_t kSchwarzMaxLds = 160 * 1024;
struct SchwarzCfg {
  int variant = kSchwarzValueFlags;
  int threads = 1024;   // threads per subdomain workgroup (a multiple of 64, at most 1024)
  int sleep = 1;        // back off with s_sleep while waiting on a dependency
};
inline size_t schwarz_value_lds(int max_rows, int nrhs, size_t elem) { return 2 * (size_t)max_rows * nrhs * elem; }
constexpr int kSchwarzValueMaxLen = 128;   // longest factor row the values-as-flags kernel takes
hipError_t launch_schwarz(const SchwarzCfg& cfg, const DevPC* pcs, const WorkItem* work, int nwork, int max_rows,
                          int max_len, int fp32, int nrhs, const double* r, double* z, hipStream_t s,
                          const Gate& gate = Gate{});

}  // namespace cpm

struct cpm_precond_s {
  const cpm_operator_s* op = nullptr;
  cpm_precond_opts opts{};
  cpm::SchwarzHost host;        // partition and sizes kept for export / info (factor arrays freed)
  cpm::DevPC P{};
  cpm::DevBuf<cpm::DevPC> d_pc;
  cpm::DevBuf<cpm::DevSub> d_subs;
  cpm::DevBuf<int32_t> d_in, d_out, d_err, d_gL;
  cpm::DevBuf<uint64_t> d_recL, d_recU;
  cpm::DevBuf<uint32_t> d_pk;
  bool packets = false;         // factor rows grouped into packets (the packet kernel runs)
  cpm::DevBuf<uint16_t> d_lcol, d_ucol;
  cpm::DevBuf<char> d_lval, d_uval, d_dinv;
  cpm::DevBuf<cpm::WorkItem> d_work;
  std::vector<cpm::WorkItem> h_work;
  int64_t serial = 0;           // identifies this preconditioner in solver caches
  cpm::SchwarzCfg cfg;          // kernel configuration (tunable)
  int max_rows = 0, max_levels = 0, max_len = 0;
  int64_t total_rows = 0, total_nnz = 0;
  // coarse level (two-level Schwarz): device arrays and the kernels' view of them
  cpm::DevCoarse C{};
  cpm::DevBuf<int32_t> d_own_ptr, d_own_idx, d_owner;
  cpm::DevBuf<double> d_ainv;
  mutable cpm::DevBuf<double> d_cv, d_ev, d_tz, d_tr;   // scratch of the single-preconditioner apply
};
