// Pieces of the sweep drivers shared by the dense and the block-sparse DMRG:
// device buffers that grow, the local eigensolver (Davidson with FP64 basis
// and matvecs at a chosen precision), the truncation rule of Sec. 5.
#pragma once

#include <chrono>
#include <functional>
#include <vector>

#include "handle.h"

struct itn_mpo {
  int32_t N = 0, w = 0, d = 0;
  std::vector<double> W;  // host, N * w*w*d*d
  const double* site(int i) const { return W.data() + (size_t)i * w * w * d * d; }
};

namespace itn {

// Device buffer that only grows.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  itn_status ensure(itn_handle* h, size_t b) {
    if (b <= bytes) return ITN_OK;
    if (p) {
      ITN_HIP(h, hipDeviceSynchronize());
      ITN_HIP(h, hipFree(p));
    }
    p = nullptr;
    bytes = 0;
    if (hipMalloc(&p, b) != hipSuccess) {
      p = nullptr;
      return fail(h, ITN_E_WORKSPACE, "allocation of %zu bytes failed", b);
    }
    bytes = b;
    return ITN_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  double* d() const { return static_cast<double*>(p); }
};

// Pinned host staging for the small device-to-host reads of the sweep
// (Davidson reductions, eigenvalues of the bond split): a read into pinned
// memory completes without the staging copy of a pageable destination.
struct HostPin {
  void* p = nullptr;
  size_t bytes = 0;
  itn_status ensure(itn_handle* h, size_t b) {
    if (b <= bytes) return ITN_OK;
    if (p) {
      ITN_HIP(h, hipDeviceSynchronize());
      ITN_HIP(h, hipHostFree(p));
    }
    p = nullptr;
    bytes = 0;
    if (hipHostMalloc(&p, b, hipHostMallocDefault) != hipSuccess) {
      p = nullptr;
      return fail(h, ITN_E_WORKSPACE, "pinned allocation of %zu bytes failed", b);
    }
    bytes = b;
    return ITN_OK;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
  }
  double* d() const { return static_cast<double*>(p); }
};


// Scratch of the local eigensolver.
struct SolverBufs {
  DBuf V, AV, partial, dots;
  HostPin pin;
  void release() {
    for (DBuf* b : {&V, &AV, &partial, &dots}) b->release();
    pin.release();
  }
};

// State of one sweep shared by the eigensolver: handle, parameters, stream,
// scratch, counters and per-phase seconds.
struct SolveCtx {
  itn_handle* h = nullptr;
  const itn_sweep_params* p = nullptr;
  hipStream_t s = nullptr;
  SolverBufs* sb = nullptr;
  int64_t matvecs = 0;    // H_eff applications (vectors), all precisions
  int64_t matvecs64 = 0;  // of which in FP64
  double max_resid = 0.0;
  bool unconverged = false;
  // per-phase seconds of the current sweep (params->timing only)
  double t_mv = 0.0, t_solve = 0.0, t_split = 0.0, t_env = 0.0;
};

// Adds the wall time of a scope to *acc when timing is on; the stream is
// drained at both ends so that the time belongs to the phase.
struct PhaseTimer {
  SolveCtx& c;
  double* acc;
  std::chrono::steady_clock::time_point t0;
  PhaseTimer(SolveCtx& ctx, double* a) : c(ctx), acc(a) {
    if (c.p->timing) {
      (void)hipStreamSynchronize(c.s);
      t0 = std::chrono::steady_clock::now();
    }
  }
  ~PhaseTimer() {
    if (c.p->timing) {
      (void)hipStreamSynchronize(c.s);
      *acc += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
  }
};

// y = H_eff x for nv vectors stored one after another (FP64 vectors of the
// solver's length), at matrix-core precision `prec`.
using Matvec = std::function<itn_status(int prec, const double* x, double* y, int nv)>;

// Lowest eigenpair by Davidson (see api_dmrg.cpp); psi in/out.
itn_status davidson(SolveCtx& c, const Matvec& mv, int prec, double tol, int maxiter, double* psi,
                    int64_t n, const double* diag, bool exact_final, double* energy, double* resid,
                    bool* converged);

// Keep count per Sec. 5 from weights sorted descending (relative to their sum).
int truncation_keep(const std::vector<double>& p_desc, double cutoff, int maxdim, int mindim,
                    double* discarded);

// Cyclic Jacobi for a small symmetric k x k matrix (row-major).
void jacobi_eigh(int k, std::vector<double> A, std::vector<double>& w, std::vector<double>& V);

}  // namespace itn
