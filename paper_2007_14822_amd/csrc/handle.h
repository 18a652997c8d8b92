// Host-side internals of libitn: the handle, workspace, error plumbing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdarg>
#include <cstdio>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/itn.h"
#include "kernels.h"

namespace itn {

// Device CSR table of a W-stage (rows = outputs, entries = inputs).
struct WTable {
  int32_t nrows = 0;
  int64_t nnz = 0;
  int32_t* row_ptr = nullptr;
  int64_t* row_off = nullptr;
  int64_t* col_off = nullptr;
  double* coef = nullptr;
  int32_t* col_idx = nullptr;  // col_off as int32 (fused epilogue tables)
  float* coef32 = nullptr;     // coef as float
  void release();
};

struct Workspace {
  void* ptr = nullptr;
  size_t size = 0;
  bool caller = false;  // memory given by itn_set_workspace (never grown or freed here)
  bool query = false;   // itn_workspace_size in progress: record the request, stop
  size_t query_bytes = 0;
};

// One timed launch (events recorded on the launch stream).
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};

}  // namespace itn

struct itn_handle {
  int device = -1;
  std::string err;
  itn::Workspace ws;
  std::map<std::string, std::unique_ptr<itn::WTable>> wtables;
  void* solver = nullptr;  // rocblas_handle for rocSOLVER, created on first use
  bool prof_on = false;
  std::vector<itn::ProfRec> prof;
  std::vector<hipEvent_t> ev_pool;
};

namespace itn {

// Status with message recorded on the handle.
itn_status fail(itn_handle* h, itn_status st, const char* fmt, ...);
itn_status hip_fail(itn_handle* h, hipError_t e, const char* where);

#define ITN_HIP(h, expr)                                   \
  do {                                                     \
    hipError_t _e = (expr);                                \
    if (_e != hipSuccess) return ::itn::hip_fail(h, _e, #expr); \
  } while (0)

#define ITN_TRY(expr)                  \
  do {                                 \
    itn_status _s = (expr);            \
    if (_s != ITN_OK) return _s;       \
  } while (0)

// Grow the handle's workspace to at least `bytes` (waits for the device).  With a
// caller workspace, fail with ITN_E_WORKSPACE if it is smaller; during a size
// query, record `bytes` and return ITN_STOP_QUERY before any work is queued.
static const itn_status ITN_STOP_QUERY = static_cast<itn_status>(1000);
itn_status ensure_workspace(itn_handle* h, size_t bytes);

// Carve 256-byte-aligned regions out of a workspace.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  void* take(size_t bytes) {
    void* p = base ? base + off : nullptr;
    off += (bytes + 255) & ~size_t(255);
    return p;
  }
};

inline size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

// Look up or build (and upload) a W-stage table keyed by its content.
itn_status get_wtable(itn_handle* h, const std::string& key, const std::vector<int32_t>& row_ptr,
                      const std::vector<int64_t>& row_off, const std::vector<int64_t>& col_off,
                      const std::vector<double>& coef, const WTable** out);

// Scoped per-kernel timer: records a pair of events around the launches in
// its scope when profiling is enabled on the handle.
struct Prof {
  itn_handle* h;
  const char* name;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  Prof(itn_handle* h_, const char* n, hipStream_t s_);
  ~Prof();
};

// A device region that scratch is carved from instead of the handle's
// workspace (nothing is allocated when one is given).
struct FixedScratch {
  void* base = nullptr;
  size_t bytes = 0;
};

// Dense H_eff of a sum of n terms (itn_heff_apply, itn_heff_apply_sum and
// the allocation-free variant); fixed = nullptr uses the handle's workspace.
itn_status heff_apply_terms(itn_handle* h, int n, const itn_tensor* const* Ls,
                            const itn_tensor* const* W1s, const itn_tensor* const* W2s,
                            const itn_tensor* const* Rs, const itn_tensor* psi, int32_t nv,
                            itn_tensor* out, itn_prec prec, void* hip_stream,
                            const FixedScratch* fixed);

// itn_contract for operands with QN index spaces (block-sparse).
itn_status contract_qn(itn_handle* h, const itn_tensor* A, const itn_tensor* B, itn_tensor* C,
                       itn_prec prec, void* hip_stream);

// Fix a QN plan's launch modes and launch it without a graph (sweeps).
itn_status qn_plan_set_direct(itn_plan* pl, int mode_stage1, int mode_stage4);
// A QN plan for the same operands at another precision, derived from `src`
// before its first apply or environment preparation (src holds no device
// state yet; ITN_E_ARG otherwise): the structure tables are copied, the
// precision-dependent lists rebuilt.  The caller owns *out.
itn_status qn_plan_at_prec(itn_handle* h, const itn_plan* src, int prec, itn_plan** out);

// Looks up the allocation-free entry point's scratch on `device` (current).
void noalloc_scratch_init(int device);

// Host-side CSR builders.
struct CSR {
  std::vector<int32_t> row_ptr{0};
  std::vector<int64_t> row_off;
  std::vector<int64_t> col_off;
  std::vector<double> coef;
  std::string key() const;
};

}  // namespace itn
