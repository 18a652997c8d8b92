// Two-site DMRG sweep driver of libitn: FP64 Davidson eigensolver with
// matrix-core matvecs, FP64 truncated bond split on rocSOLVER, environment
// updates, sweep schedule (the DMRG algorithm of Sec. 7.2 with the
// truncation of Sec. 5).
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "common.h"
#include "handle.h"

using namespace itn;

struct itn_mpo {
  int32_t N = 0, w = 0, d = 0;
  std::vector<double> W;  // host, N * w*w*d*d
  const double* site(int i) const { return W.data() + (size_t)i * w * w * d * d; }
};

namespace {

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

}  // namespace

struct itn_mps {
  int32_t N = 0, d = 0;
  std::vector<int32_t> bond;   // N+1
  std::vector<DBuf> site;      // N, FP64 [bond[i], d, bond[i+1]]
  std::vector<DBuf> Lenv;      // N+1: Lenv[k] = environment of sites [0, k)
  std::vector<DBuf> Renv;      // N+1: Renv[k] = environment of sites [k, N)
  bool envs = false;
  int mpo_w = 0;
  // overlap environments with the states of an excited-state sweep:
  // OL[j][k] = <psi|phi_j> over sites [0, k), OR[j][k] over [k, N)
  std::vector<std::vector<DBuf>> OL, OR;
  // driver scratch
  DBuf psi, tmp, rho, evec, eval, einfo, V, AV, Lp, Rp, partial, dots, ev_host_stage;
  DBuf ovec, ot1, ot2, ot3, odots;
  DBuf hh, hscr;  // bond split: Householder reflectors [n][n]; tridiagonal and barrier scratch
  HostPin pin;    // pinned host staging for small reads
  ~itn_mps() {
    for (auto& b : site) b.release();
    for (auto& b : Lenv) b.release();
    for (auto& b : Renv) b.release();
    for (auto* v : {&OL, &OR})
      for (auto& row : *v)
        for (auto& b : row) b.release();
    for (DBuf* b : {&psi, &tmp, &rho, &evec, &eval, &einfo, &V, &AV, &Lp, &Rp, &partial, &dots,
                    &ev_host_stage, &ovec, &ot1, &ot2, &ot3, &odots, &hh, &hscr})
      b->release();
    pin.release();
  }
};

extern "C" void itn_release_solver(itn_handle* h) {
  if (h && h->solver) {
    rocblas_destroy_handle(static_cast<rocblas_handle>(h->solver));
    h->solver = nullptr;
  }
}

namespace {

// ------------------------------------------------------------ small eigh
// Cyclic Jacobi for a symmetric k x k matrix (row-major); eigenvalues
// ascending in w, eigenvectors as the columns of V (row-major k x k).
void jacobi_eigh(int k, std::vector<double> A, std::vector<double>& w, std::vector<double>& V) {
  V.assign((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) V[i * k + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        tot += A[i * k + j] * A[i * k + j];
        if (i != j) off += A[i * k + j] * A[i * k + j];
      }
    if (off <= 1e-32 * std::max(tot, 1e-300)) break;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = A[p * k + q];
        if (apq == 0.0) continue;
        const double app = A[p * k + p], aqq = A[q * k + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < k; ++r) {  // A <- A J (columns p, q)
          const double arp = A[r * k + p], arq = A[r * k + q];
          A[r * k + p] = c * arp - s * arq;
          A[r * k + q] = s * arp + c * arq;
        }
        for (int r = 0; r < k; ++r) {  // A <- J^T A (rows p, q)
          const double apr = A[p * k + r], aqr = A[q * k + r];
          A[p * k + r] = c * apr - s * aqr;
          A[q * k + r] = s * apr + c * aqr;
        }
        for (int r = 0; r < k; ++r) {
          const double vrp = V[r * k + p], vrq = V[r * k + q];
          V[r * k + p] = c * vrp - s * vrq;
          V[r * k + q] = s * vrp + c * vrq;
        }
      }
  }
  std::vector<int> idx(k);
  for (int i = 0; i < k; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return A[a * k + a] < A[b * k + b]; });
  w.resize(k);
  std::vector<double> V2((size_t)k * k);
  for (int j = 0; j < k; ++j) {
    w[j] = A[idx[j] * k + idx[j]];
    for (int r = 0; r < k; ++r) V2[r * k + j] = V[r * k + idx[j]];
  }
  V.swap(V2);
}

itn_tensor dense_t(int rank, const int64_t* dims, itn_dtype dt, void* data) {
  itn_tensor t{};
  t.rank = rank;
  t.dims = dims;
  t.dtype = dt;
  t.data = data;
  return t;
}

// C[M,N] = A[M,K] * B[N,K]^T, FP64 operands and output.
hipError_t gemm64(const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                  int64_t M, int64_t N, int64_t K, hipStream_t s) {
  GemmArgs g{};
  g.A = A;
  g.B = B;
  g.C = C;
  g.M = M;
  g.N = N;
  g.K = K;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.batch = 1;
  return gemm_nt(P_F64, D_F64, g, s);
}

// out[c][r] = in[r][c] for an rows x cols FP64 matrix.
hipError_t transpose64(const double* in, double* out, int64_t rows, int64_t cols, hipStream_t s) {
  TransposeArgs t{};
  t.rows = rows;
  t.cols = cols;
  t.nzb = 1;
  t.nzc = 1;
  t.in_r = cols;
  t.in_c = 1;
  t.out_c = rows;
  t.out_r = 1;
  return transpose_cast(D_F64, in, D_F64, out, t, s);
}

struct Ctx {
  itn_handle* h;
  itn_mps* m;
  const itn_mpo* mpo;
  const itn_sweep_params* p;
  hipStream_t s = nullptr;
  int64_t matvecs = 0;
  double max_resid = 0.0;
  bool unconverged = false;
  // per-phase seconds of the current sweep (params->timing only)
  double t_mv = 0.0, t_solve = 0.0, t_split = 0.0, t_env = 0.0;
  // excited states: projected previous states at the current bond
  int northo = 0;
  const double* pen_v = nullptr;  // northo vectors of the bond's length
};

// Adds the wall time of a scope to *acc when timing is on; the stream is
// drained at both ends so that the time belongs to the phase.
struct PhaseTimer {
  Ctx& c;
  double* acc;
  std::chrono::steady_clock::time_point t0;
  PhaseTimer(Ctx& ctx, double* a) : c(ctx), acc(a) {
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

// y = H_eff x at precision `prec` (FP64 vectors), through the public entry point.
itn_status heff(Ctx& c, int i, int prec, const double* x, double* y, int64_t cl, int64_t cr) {
  PhaseTimer pt(c, &c.t_mv);
  const int w = c.mpo->w, d = c.mpo->d;
  const int64_t dl[3] = {cl, w, cl}, dr[3] = {cr, w, cr}, dw[4] = {w, w, d, d};
  const int64_t dp[4] = {cl, d, d, cr};
  const bool low = prec != ITN_P_F64;
  const itn_dtype et = prec == ITN_P_BF16 ? ITN_BF16 : (prec == ITN_P_F32 ? ITN_F32 : ITN_F64);
  itn_tensor L = dense_t(3, dl, et, low ? c.m->Lp.p : c.m->Lenv[i].p);
  itn_tensor R = dense_t(3, dr, et, low ? c.m->Rp.p : c.m->Renv[i + 2].p);
  itn_tensor W1 = dense_t(4, dw, ITN_F64, const_cast<double*>(c.mpo->site(i)));
  itn_tensor W2 = dense_t(4, dw, ITN_F64, const_cast<double*>(c.mpo->site(i + 1)));
  itn_tensor P = dense_t(4, dp, ITN_F64, const_cast<double*>(x));
  itn_tensor O = dense_t(4, dp, ITN_F64, y);
  c.matvecs++;
  ITN_TRY(itn_heff_apply(c.h, &L, &W1, &W2, &R, &P, 1, &O, (itn_prec)prec, c.s));
  if (c.northo > 0) {  // + weight * sum_j |v_j><v_j| x  (Sec. 7.2 energy penalty)
    const int64_t n = cl * d * d * cr;
    ITN_TRY(c.m->partial.ensure(c.h, (size_t)c.northo * dot_blocks(n) * 8));
    ITN_TRY(c.m->odots.ensure(c.h, (size_t)c.northo * 8 + 8));
    ITN_HIP(c.h, multi_dot(c.pen_v, n, c.northo, x, n, c.m->partial.d(), c.m->odots.d(), c.s));
    ITN_HIP(c.h, lincomb_dev(c.pen_v, n, c.northo, c.m->odots.d(), c.p->weight, y, n, c.s));
  }
  return ITN_OK;
}

// <V_j, w> for j < k, to host.
itn_status dots(Ctx& c, const double* V, int64_t n, int k, const double* w, double* out) {
  ITN_TRY(c.m->partial.ensure(c.h, (size_t)k * dot_blocks(n) * 8));
  ITN_TRY(c.m->dots.ensure(c.h, (size_t)k * 8 + 8));
  ITN_TRY(c.m->pin.ensure(c.h, (size_t)k * 8 + 8));
  ITN_HIP(c.h, multi_dot(V, n, k, w, n, c.m->partial.d(), c.m->dots.d(), c.s));
  ITN_HIP(c.h, hipMemcpyAsync(c.m->pin.p, c.m->dots.p, (size_t)k * 8, hipMemcpyDeviceToHost, c.s));
  ITN_HIP(c.h, hipStreamSynchronize(c.s));
  std::memcpy(out, c.m->pin.p, (size_t)k * 8);
  return ITN_OK;
}

// Lowest eigenpair of H_eff at bond i by Davidson (identity preconditioner,
// full re-orthogonalisation, thick restart), FP64 vectors.  psi (in/out,
// length n) is the start vector and the result.  *converged is false only
// when maxiter matvecs ended above the tolerance; a residual already inside
// the Krylov space (no new direction) is at the arithmetic's noise floor and
// counts as converged.
//
// Host round trips per expansion step: two, sometimes three.  (1) the new
// column V^T A v_k of the projected matrix; (2) V^T r and r.r in one
// reduction, the residual being formed in the next basis slot; (3) only when
// the first Gram-Schmidt pass removed most of r (DGKS test): the same pair
// after that pass, from which the norm after the second pass follows as
// |r'|^2 - |c2|^2 (V orthonormal).
itn_status davidson(Ctx& c, int i, int prec, double tol, int maxiter, double* psi, int64_t n,
                    int64_t cl, int64_t cr, double* energy, double* resid, bool* converged) {
  const int kmax = std::max(4, std::min(c.p->krylovdim, 32));
  constexpr int KEEP = 3;  // Ritz vectors kept at a restart (thick restart)
  ITN_TRY(c.m->V.ensure(c.h, (size_t)(kmax + KEEP) * n * 8));
  ITN_TRY(c.m->AV.ensure(c.h, (size_t)(kmax + KEEP) * n * 8));
  double* V = c.m->V.d();
  double* AV = c.m->AV.d();
  std::vector<double> Hk((size_t)kmax * kmax, 0.0), tmp(kmax + 2);
  double nrm2;
  ITN_TRY(dots(c, psi, n, 1, psi, &nrm2));
  if (!(nrm2 > 0)) return fail(c.h, ITN_E_ARG, "zero start vector at bond %d", i);
  ITN_HIP(c.h, hipMemcpyAsync(V, psi, n * 8, hipMemcpyDeviceToDevice, c.s));
  ITN_HIP(c.h, scale(V, 1.0 / std::sqrt(nrm2), n, c.s));
  ITN_TRY(heff(c, i, prec, V, AV, cl, cr));
  int k = 1;
  double theta = 0.0, rn = 0.0;
  bool conv = false;
  std::vector<double> w, Y, y;
  for (int it = 0;; ++it) {
    // (1) new column k-1 of the projected matrix
    ITN_TRY(dots(c, V, n, k, AV + (size_t)(k - 1) * n, tmp.data()));
    for (int a = 0; a < k; ++a) {
      Hk[a * kmax + (k - 1)] = tmp[a];
      Hk[(k - 1) * kmax + a] = tmp[a];
    }
    std::vector<double> Hs((size_t)k * k);
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b) Hs[a * k + b] = 0.5 * (Hk[a * kmax + b] + Hk[b * kmax + a]);
    jacobi_eigh(k, Hs, w, Y);
    theta = w[0];
    y.assign(k, 0.0);
    for (int a = 0; a < k; ++a) y[a] = Y[a * k + 0];
    if (k == kmax) {  // thick restart from the lowest KEEP Ritz vectors
      const int keep = std::min(KEEP, k - 1);
      for (int j = 0; j < keep; ++j) {
        std::vector<double> yj(k);
        for (int a = 0; a < k; ++a) yj[a] = Y[a * k + j];
        ITN_HIP(c.h, lincomb(V, n, k, yj.data(), 0.0, V + (size_t)(kmax + j) * n, n, c.s));
        ITN_HIP(c.h, lincomb(AV, n, k, yj.data(), 0.0, AV + (size_t)(kmax + j) * n, n, c.s));
      }
      ITN_HIP(c.h, hipMemcpyAsync(V, V + (size_t)kmax * n, (size_t)keep * n * 8,
                                  hipMemcpyDeviceToDevice, c.s));
      ITN_HIP(c.h, hipMemcpyAsync(AV, AV + (size_t)kmax * n, (size_t)keep * n * 8,
                                  hipMemcpyDeviceToDevice, c.s));
      std::fill(Hk.begin(), Hk.end(), 0.0);
      for (int j = 0; j < keep; ++j) Hk[j * kmax + j] = w[j];
      k = keep;
      y.assign(k, 0.0);
      y[0] = 1.0;
    }
    // r = AV y - theta V y, in slot k (the next basis vector if r is kept)
    double* r = V + (size_t)k * n;
    std::vector<double> ny(k);
    for (int a = 0; a < k; ++a) ny[a] = -theta * y[a];
    ITN_HIP(c.h, lincomb(AV, n, k, y.data(), 0.0, r, n, c.s));
    ITN_HIP(c.h, lincomb(V, n, k, ny.data(), 1.0, r, n, c.s));
    // (2) V^T r and r.r
    ITN_TRY(dots(c, V, n, k + 1, r, tmp.data()));
    const double r2 = tmp[k];
    rn = std::sqrt(std::max(r2, 0.0));
    if (rn <= tol * std::max(1.0, std::fabs(theta))) {
      conv = true;
      break;
    }
    if (it + 1 >= maxiter) break;
    // Gram-Schmidt against V.  With V orthonormal the projected norm is
    // r.r - |V^T r|^2; a second pass (and its reduction) is needed only when
    // the projection removed much of r (Daniel-Gragg-Kaufman-Stewart test:
    // kept norm below 1/sqrt(2)).  The Galerkin residual is orthogonal to V
    // up to rounding, so one pass is the common case.
    double p2 = 0.0;
    for (int a = 0; a < k; ++a) {
      p2 += tmp[a] * tmp[a];
      tmp[a] = -tmp[a];
    }
    ITN_HIP(c.h, lincomb(V, n, k, tmp.data(), 1.0, r, n, c.s));
    double t2 = r2 - p2;
    if (!(t2 > 0.5 * r2)) {
      ITN_TRY(dots(c, V, n, k + 1, r, tmp.data()));  // (3) second pass
      double c2 = 0.0;
      for (int a = 0; a < k; ++a) {
        c2 += tmp[a] * tmp[a];
        tmp[a] = -tmp[a];
      }
      t2 = tmp[k] - c2;
      if (!(t2 > 1e-28 * std::max(1.0, r2))) {  // no new direction
        conv = true;
        break;
      }
      ITN_HIP(c.h, lincomb(V, n, k, tmp.data(), 1.0, r, n, c.s));
    }
    ITN_HIP(c.h, scale(r, 1.0 / std::sqrt(t2), n, c.s));
    ITN_TRY(heff(c, i, prec, r, AV + (size_t)k * n, cl, cr));
    ++k;
  }
  // the Ritz vector of the last projected problem
  ITN_HIP(c.h, lincomb(V, n, k, y.data(), 0.0, psi, n, c.s));
  *energy = theta;
  *resid = rn;
  *converged = conv;
  return ITN_OK;
}

rocblas_handle solver(Ctx& c) {
  if (!c.h->solver) {
    rocblas_handle r = nullptr;
    if (rocblas_create_handle(&r) != rocblas_status_success) return nullptr;
    c.h->solver = r;
  }
  rocblas_handle r = static_cast<rocblas_handle>(c.h->solver);
  rocblas_set_stream(r, c.s);
  return r;
}

// Keep count per Sec. 5: discard the smallest weights while their running sum
// stays within the cutoff, cap at maxdim, keep at least mindim (and one).
int truncation_keep(const std::vector<double>& p_desc, double cutoff, int maxdim, int mindim,
                    double* discarded) {
  const int n = (int)p_desc.size();
  int keep = n;
  double disc = 0.0;
  while (keep > 1 && disc + p_desc[keep - 1] <= cutoff) {
    disc += p_desc[keep - 1];
    --keep;
  }
  keep = std::min(keep, maxdim);
  keep = std::max(keep, std::min(std::max(mindim, 1), n));
  double d = 0.0;
  for (int j = keep; j < n; ++j) d += p_desc[j];
  *discarded = d;
  return keep;
}

// ITN_EIG=library selects rocSOLVER's full symmetric eigensolver for every
// bond split (comparison runs); default is the cooperative tridiagonalisation.
bool use_coop_sytrd() {
  const char* e = std::getenv("ITN_EIG");
  return !(e && std::strcmp(e, "library") == 0);
}

// Split psi [cl, d, d, cr] at bond i and store the new sites i, i+1.
itn_status split(Ctx& c, int i, bool to_right, int64_t cl, int64_t cr, int maxdim, double cutoff,
                 double* trunc) {
  itn_mps* m = c.m;
  const int d = c.m->d;
  const int64_t nl = cl * d, nr = cr * d;  // M is nl x nr
  const int64_t n = to_right ? nl : nr;    // density-matrix dimension
  double* M = m->psi.d();
  ITN_TRY(m->tmp.ensure(c.h, (size_t)nl * nr * 8));
  ITN_TRY(m->rho.ensure(c.h, (size_t)n * n * 8));
  ITN_TRY(m->eval.ensure(c.h, (size_t)n * 2 * 8));
  ITN_TRY(m->einfo.ensure(c.h, 64));
  double* MT = m->tmp.d();
  ITN_HIP(c.h, transpose64(M, MT, nl, nr, c.s));  // MT [nr][nl]
  double* rho = m->rho.d();
  if (to_right) ITN_HIP(c.h, gemm64(M, nr, M, nr, rho, n, n, n, nr, c.s));      // M M^T
  else ITN_HIP(c.h, gemm64(MT, nl, MT, nl, rho, n, n, n, nl, c.s));             // M^T M
  rocblas_handle rb = solver(c);
  if (!rb) return fail(c.h, ITN_E_HIP, "rocblas handle creation failed");
  double* D = m->eval.d();
  double* E = D + n;
  std::vector<double> ev(n);
  rocblas_int info = 0;
  // Eigen-decomposition of rho.  Householder tridiagonalisation in one
  // cooperative launch, the tridiagonal eigenproblem by rocSOLVER's divide
  // and conquer, the kept eigenvectors back-transformed; the library's full
  // symmetric solver where n does not fit (or ITN_EIG=library).
  const int nwg = use_coop_sytrd() && tridiag_back_supported((int)n) ? sytrd_coop_groups((int)n) : 0;
  bool coop = nwg > 0;
  double *hhV = nullptr, *tau = nullptr;
  int* coop_err = nullptr;
  if (coop) {
    ITN_TRY(m->hh.ensure(c.h, (size_t)n * n * 8));
    ITN_TRY(m->hscr.ensure(c.h, (size_t)(5 * n + 2 * nwg + 8) * 8));
    hhV = m->hh.d();
    double* scr = m->hscr.d();
    tau = scr;
    SytrdArgs sa{};
    sa.A = rho;
    sa.lda = n;
    sa.n = (int)n;
    sa.nwg = nwg;
    sa.d = D;
    sa.e = E;
    sa.tau = tau;
    sa.V = hhV;
    sa.pub = scr + n;
    sa.pbuf = scr + 3 * n;
    sa.dots = scr + 5 * n;
    sa.bar = reinterpret_cast<unsigned*>(scr + 5 * n + 2 * nwg);
    sa.err = reinterpret_cast<int*>(scr + 5 * n + 2 * nwg + 1);
    sa.spin_limit = (int64_t)1 << 24;
    coop_err = sa.err;
    if (sytrd_coop(sa, c.s) != hipSuccess) {  // e.g. no cooperative launch: library path
      (void)hipGetLastError();
      coop = false;
    }
  }
  if (coop) {
    // eigenvectors of T into rho's storage (column j: eigenvalue j, ascending)
    rocblas_status st = rocsolver_dstedc(rb, rocblas_evect_tridiagonal, (rocblas_int)n, D, E, rho,
                                         (rocblas_int)n, static_cast<rocblas_int*>(m->einfo.p));
    if (st != rocblas_status_success) return fail(c.h, ITN_E_HIP, "rocsolver_dstedc failed (%d)", (int)st);
    int err = 0;
    ITN_TRY(m->pin.ensure(c.h, (size_t)(n + 2) * 8));
    char* pin = static_cast<char*>(m->pin.p);
    ITN_HIP(c.h, hipMemcpyAsync(pin, D, n * 8, hipMemcpyDeviceToHost, c.s));
    ITN_HIP(c.h, hipMemcpyAsync(pin + n * 8, m->einfo.p, sizeof(info), hipMemcpyDeviceToHost, c.s));
    ITN_HIP(c.h, hipMemcpyAsync(pin + (n + 1) * 8, coop_err, sizeof(err), hipMemcpyDeviceToHost, c.s));
    ITN_HIP(c.h, hipStreamSynchronize(c.s));
    std::memcpy(ev.data(), pin, n * 8);
    std::memcpy(&info, pin + n * 8, sizeof(info));
    std::memcpy(&err, pin + (n + 1) * 8, sizeof(err));
    if (err != 0) {  // a grid barrier gave up: redo this bond with the library solver
      coop = false;
      if (to_right) ITN_HIP(c.h, gemm64(M, nr, M, nr, rho, n, n, n, nr, c.s));
      else ITN_HIP(c.h, gemm64(MT, nl, MT, nl, rho, n, n, n, nl, c.s));
    }
  }
  if (!coop) {
    rocblas_status st = rocsolver_dsyevd(rb, rocblas_evect_original, rocblas_fill_upper, (rocblas_int)n,
                                         rho, (rocblas_int)n, D, E,
                                         static_cast<rocblas_int*>(m->einfo.p));
    if (st != rocblas_status_success) return fail(c.h, ITN_E_HIP, "rocsolver_dsyevd failed (%d)", (int)st);
    ITN_TRY(m->pin.ensure(c.h, (size_t)(n + 2) * 8));
    char* pin = static_cast<char*>(m->pin.p);
    ITN_HIP(c.h, hipMemcpyAsync(pin, D, n * 8, hipMemcpyDeviceToHost, c.s));
    ITN_HIP(c.h, hipMemcpyAsync(pin + n * 8, m->einfo.p, sizeof(info), hipMemcpyDeviceToHost, c.s));
    ITN_HIP(c.h, hipStreamSynchronize(c.s));
    std::memcpy(ev.data(), pin, n * 8);
    std::memcpy(&info, pin + n * 8, sizeof(info));
  }
  if (info != 0) return fail(c.h, ITN_E_NOT_CONVERGED, "symmetric eigensolver info=%d at bond %d", (int)info, i);
  // Weights, descending.  The n x n density matrix of the nl x nr matrix M
  // has rank at most min(nl, nr): its spectrum beyond that is structurally
  // zero (rounding noise of either sign), and the truncated SVD of Sec. 5 has
  // only min(nl, nr) singular values to keep, so only those enter.
  const int64_t nsv = std::min(nl, nr);
  std::vector<double> pd(nsv);
  double tot = 0.0;
  for (int64_t j = 0; j < nsv; ++j) {
    pd[j] = std::max(ev[n - 1 - j], 0.0);
    tot += pd[j];
  }
  if (!(tot > 0)) return fail(c.h, ITN_E_ARG, "zero two-site state at bond %d", i);
  for (auto& x : pd) x /= tot;
  const int k = truncation_keep(pd, cutoff, maxdim, c.p->mindim, trunc);
  double kept = 0.0;
  for (int j = 0; j < k; ++j) kept += pd[j] * tot;
  const double inv = 1.0 / std::sqrt(kept);
  // Uk^T: row r = eigenvector of the r-th largest eigenvalue
  ITN_TRY(m->evec.ensure(c.h, (size_t)k * n * 8));
  double* Ukt = m->evec.d();
  if (coop) {
    ITN_HIP(c.h, tridiag_back(hhV, tau, rho, n, (int)n - 1, Ukt, (int)n, k, c.s));
  } else {
    // column j of rho holds eigenvector j: copy n-k .. n-1, then reverse the row order
    ITN_HIP(c.h, hipMemcpy2DAsync(Ukt, n * 8, rho + (size_t)(n - k) * n, n * 8, n * 8, k,
                                  hipMemcpyDeviceToDevice, c.s));
    const int64_t dims[2] = {k, n};
    const int64_t strides[2] = {-n, 1};
    ITN_TRY(m->Lp.ensure(c.h, (size_t)k * n * 8));  // scratch before the next bond
    ITN_HIP(c.h, permute_cast(D_F64, Ukt + (size_t)(k - 1) * n, D_F64, m->Lp.p, 2, dims, strides, c.s));
    ITN_HIP(c.h, hipMemcpyAsync(Ukt, m->Lp.p, (size_t)k * n * 8, hipMemcpyDeviceToDevice, c.s));
  }
  DBuf& Sa = m->site[i];
  DBuf& Sb = m->site[i + 1];
  ITN_TRY(Sa.ensure(c.h, (size_t)cl * d * k * 8));
  ITN_TRY(Sb.ensure(c.h, (size_t)k * d * cr * 8));
  if (to_right) {
    // A_i[(a s1), j] = U[(a s1), j];  A_{i+1}[j, (s2 b)] = (U^T M)[j, (s2 b)] / |S_k|
    ITN_HIP(c.h, transpose64(Ukt, Sa.d(), k, nl, c.s));
    ITN_HIP(c.h, gemm64(Ukt, nl, MT, nl, Sb.d(), nr, k, nr, nl, c.s));
    ITN_HIP(c.h, scale(Sb.d(), inv, (int64_t)k * nr, c.s));
  } else {
    // A_{i+1}[j, (s2 b)] = V^T[j, (s2 b)];  A_i[(a s1), j] = (M V)[(a s1), j] / |S_k|
    ITN_HIP(c.h, hipMemcpyAsync(Sb.p, Ukt, (size_t)k * nr * 8, hipMemcpyDeviceToDevice, c.s));
    ITN_HIP(c.h, gemm64(M, nr, Ukt, nr, Sa.d(), k, nl, k, nr, c.s));
    ITN_HIP(c.h, scale(Sa.d(), inv, nl * (int64_t)k, c.s));
  }
  m->bond[i + 1] = k;
  return ITN_OK;
}

itn_status env_step(Ctx& c, int i, bool left) {
  itn_mps* m = c.m;
  const int w = c.mpo->w, d = m->d;
  const int64_t dw[4] = {w, w, d, d};
  itn_tensor Wt = dense_t(4, dw, ITN_F64, const_cast<double*>(c.mpo->site(i)));
  if (left) {  // Lenv[i+1] from Lenv[i] and site i
    const int64_t a = m->bond[i], b = m->bond[i + 1];
    const int64_t de[3] = {a, w, a}, da[3] = {a, d, b}, doo[3] = {b, w, b};
    ITN_TRY(m->Lenv[i + 1].ensure(c.h, (size_t)b * w * b * 8));
    itn_tensor E = dense_t(3, de, ITN_F64, m->Lenv[i].p);
    itn_tensor A = dense_t(3, da, ITN_F64, m->site[i].p);
    itn_tensor O = dense_t(3, doo, ITN_F64, m->Lenv[i + 1].p);
    return itn_env_update(c.h, &E, &A, &Wt, ITN_LEFT, &O, ITN_P_F64, c.s);
  }
  // Renv[i] from Renv[i+1] and site i
  const int64_t a = m->bond[i], b = m->bond[i + 1];
  const int64_t de[3] = {b, w, b}, da[3] = {a, d, b}, doo[3] = {a, w, a};
  ITN_TRY(m->Renv[i].ensure(c.h, (size_t)a * w * a * 8));
  itn_tensor E = dense_t(3, de, ITN_F64, m->Renv[i + 1].p);
  itn_tensor A = dense_t(3, da, ITN_F64, m->site[i].p);
  itn_tensor O = dense_t(3, doo, ITN_F64, m->Renv[i].p);
  return itn_env_update(c.h, &E, &A, &Wt, ITN_RIGHT, &O, ITN_P_F64, c.s);
}

itn_status boundary(Ctx& c, DBuf& b, int channel) {
  const int w = c.mpo->w;
  ITN_TRY(b.ensure(c.h, (size_t)w * 8));
  std::vector<double> v(w, 0.0);
  v[channel] = 1.0;
  ITN_HIP(c.h, hipMemcpy(b.p, v.data(), w * 8, hipMemcpyHostToDevice));
  return ITN_OK;
}

// Overlap environment steps and projected states of the excited-state sweep
// (previous state phi with bonds clp, crp; psi's site A with cl, cr).
// Left:  out[b', b]  = sum_{a', s} A[a', s, b'] sum_a LO[a', a] B[a, s, b]
itn_status ov_left(Ctx& c, const double* LO, const double* A, const double* B, int64_t cl, int64_t cr,
                   int64_t clp, int64_t crp, double* out) {
  itn_mps* m = c.m;
  const int64_t d = m->d;
  // ot1 holds Bt [(s b)][a], then Tt [b][(a' s)]
  ITN_TRY(m->ot1.ensure(c.h, (size_t)std::max(d * crp * clp, cl * d * crp) * 8 + 8));
  ITN_TRY(m->ot2.ensure(c.h, (size_t)(cl * d * crp) * 8 + 8));
  ITN_TRY(m->ot3.ensure(c.h, (size_t)(cr * cl * d) * 8 + 8));
  ITN_HIP(c.h, transpose64(B, m->ot1.d(), clp, d * crp, c.s));                       // Bt[(s b)][a]
  ITN_HIP(c.h, gemm64(LO, clp, m->ot1.d(), clp, m->ot2.d(), d * crp, cl, d * crp, clp, c.s));  // T[a'][(s b)]
  ITN_HIP(c.h, transpose64(m->ot2.d(), m->ot1.d(), cl * d, crp, c.s));              // Tt[b][(a' s)]
  ITN_HIP(c.h, transpose64(A, m->ot3.d(), cl * d, cr, c.s));                        // At[b'][(a' s)]
  ITN_HIP(c.h, gemm64(m->ot3.d(), cl * d, m->ot1.d(), cl * d, out, crp, cr, crp, cl * d, c.s));
  return ITN_OK;
}
// Right: out[a', a] = sum_{s, b'} A[a', s, b'] sum_b RO[b', b] B[a, s, b]
itn_status ov_right(Ctx& c, const double* RO, const double* A, const double* B, int64_t cl, int64_t cr,
                    int64_t clp, int64_t crp, double* out) {
  itn_mps* m = c.m;
  const int64_t d = m->d;
  ITN_TRY(m->ot1.ensure(c.h, (size_t)(clp * d * cr) * 8 + 8));
  ITN_HIP(c.h, gemm64(B, crp, RO, crp, m->ot1.d(), cr, clp * d, cr, crp, c.s));     // U[(a s)][b']
  ITN_HIP(c.h, gemm64(A, d * cr, m->ot1.d(), d * cr, out, clp, cl, clp, d * cr, c.s));
  return ITN_OK;
}
// v[a', s1, s2, b'] = sum LO[a', a] B1[a, s1, m] B2[m, s2, b] RO[b', b]
itn_status ov_project(Ctx& c, const double* LO, const double* B1, const double* B2, const double* RO,
                      int64_t cl, int64_t cr, int64_t clp, int64_t mp, int64_t crp, double* out) {
  itn_mps* m = c.m;
  const int64_t d = m->d;
  ITN_TRY(m->ot1.ensure(c.h, (size_t)std::max(d * mp * clp, d * crp * mp) * 8 + 8));
  ITN_TRY(m->ot2.ensure(c.h, (size_t)(cl * d * mp) * 8 + 8));
  ITN_TRY(m->ot3.ensure(c.h, (size_t)(cl * d * d * crp) * 8 + 8));
  ITN_HIP(c.h, transpose64(B1, m->ot1.d(), clp, d * mp, c.s));                      // B1t[(s1 m)][a]
  ITN_HIP(c.h, gemm64(LO, clp, m->ot1.d(), clp, m->ot2.d(), d * mp, cl, d * mp, clp, c.s));  // P1[(a' s1)][m]
  ITN_HIP(c.h, transpose64(B2, m->ot1.d(), mp, d * crp, c.s));                      // B2t[(s2 b)][m]
  ITN_HIP(c.h, gemm64(m->ot2.d(), mp, m->ot1.d(), mp, m->ot3.d(), d * crp, cl * d, d * crp, mp, c.s));
  ITN_HIP(c.h, gemm64(m->ot3.d(), crp, RO, crp, out, cr, cl * d * d, cr, crp, c.s));
  return ITN_OK;
}

// One bond: form psi, eigensolve, split, extend the environment.
itn_status bond_step(Ctx& c, int i, bool to_right, int maxdim, double cutoff, double* energy,
                     double* trunc) {
  itn_mps* m = c.m;
  const int d = m->d;
  const int64_t cl = m->bond[i], cm = m->bond[i + 1], cr = m->bond[i + 2];
  const int64_t n = cl * d * d * cr;
  ITN_TRY(m->psi.ensure(c.h, (size_t)n * 8));
  ITN_TRY(m->tmp.ensure(c.h, (size_t)std::max<int64_t>(n, cm * d * cr) * 8));
  // psi[(a s1), (s2 b)] = A_i[(a s1), m] A_{i+1}[m, (s2 b)]
  ITN_HIP(c.h, transpose64(m->site[i + 1].d(), m->tmp.d(), cm, d * cr, c.s));
  ITN_HIP(c.h, gemm64(m->site[i].d(), cm, m->tmp.d(), cm, m->psi.d(), d * cr, cl * d, d * cr, cm, c.s));
  // operands in the matvec precision, once per bond
  const int prec = c.p->prec;
  if (prec != ITN_P_F64) {
    const int dt = prec == ITN_P_BF16 ? D_BF16 : D_F32;
    const int w = c.mpo->w;
    ITN_TRY(m->Lp.ensure(c.h, (size_t)cl * w * cl * 4 + 256));
    ITN_TRY(m->Rp.ensure(c.h, (size_t)cr * w * cr * 4 + 256));
    ITN_HIP(c.h, cast(D_F64, m->Lenv[i].p, dt, m->Lp.p, cl * w * cl, c.s));
    ITN_HIP(c.h, cast(D_F64, m->Renv[i + 2].p, dt, m->Rp.p, cr * w * cr, c.s));
  }
  if (c.northo > 0) {  // previous states seen from this bond
    ITN_TRY(m->ovec.ensure(c.h, (size_t)c.northo * n * 8));
    for (int j = 0; j < c.northo; ++j) {
      const itn_mps* o = c.p->ortho[j];
      ITN_TRY(ov_project(c, m->OL[j][i].d(), o->site[i].d(), o->site[i + 1].d(), m->OR[j][i + 2].d(), cl,
                         cr, o->bond[i], o->bond[i + 1], o->bond[i + 2], m->ovec.d() + (size_t)j * n));
    }
    c.pen_v = m->ovec.d();
  }
  const double tol = c.p->eig_tol > 0 ? c.p->eig_tol : 1e-10;
  const int maxiter = c.p->maxiter > 0 ? c.p->maxiter : 100;
  double e = 0.0, r = 0.0;
  bool conv = true;
  {
    PhaseTimer pt(c, &c.t_solve);
    if (prec == ITN_P_F64) {
      ITN_TRY(davidson(c, i, ITN_P_F64, tol, maxiter, m->psi.d(), n, cl, cr, &e, &r, &conv));
    } else {
      // low-precision phase to its own noise floor, then FP64 refinement
      const double tol_lo = std::max(tol, prec == ITN_P_BF16 ? 2e-2 : 2e-5);
      ITN_TRY(davidson(c, i, prec, tol_lo, maxiter, m->psi.d(), n, cl, cr, &e, &r, &conv));
      if (c.p->refine)
        ITN_TRY(davidson(c, i, ITN_P_F64, tol, maxiter, m->psi.d(), n, cl, cr, &e, &r, &conv));
    }
  }
  c.max_resid = std::max(c.max_resid, r);
  if (!conv && (prec == ITN_P_F64 || c.p->refine)) c.unconverged = true;
  *energy = e;
  {
    PhaseTimer pt(c, &c.t_split);
    ITN_TRY(split(c, i, to_right, cl, cr, maxdim, cutoff, trunc));
  }
  PhaseTimer pt(c, &c.t_env);
  if (to_right) ITN_TRY(env_step(c, i, true));
  else ITN_TRY(env_step(c, i + 1, false));
  for (int j = 0; j < c.northo; ++j) {  // overlap environments follow the new sites
    const itn_mps* o = c.p->ortho[j];
    const int k = to_right ? i : i + 1;
    const int64_t ocl = m->bond[k], ocr = m->bond[k + 1], pcl = o->bond[k], pcr = o->bond[k + 1];
    if (to_right) {
      ITN_TRY(m->OL[j][k + 1].ensure(c.h, (size_t)(ocr * pcr) * 8));
      ITN_TRY(ov_left(c, m->OL[j][k].d(), m->site[k].d(), o->site[k].d(), ocl, ocr, pcl, pcr,
                      m->OL[j][k + 1].d()));
    } else {
      ITN_TRY(m->OR[j][k].ensure(c.h, (size_t)(ocl * pcl) * 8));
      ITN_TRY(ov_right(c, m->OR[j][k + 1].d(), m->site[k].d(), o->site[k].d(), ocl, ocr, pcl, pcr,
                       m->OR[j][k].d()));
    }
  }
  return ITN_OK;
}

}  // namespace

// ------------------------------------------------------------------- ABI
extern "C" {

itn_status itn_mpo_create(itn_handle* h, int32_t N, int32_t w, int32_t d, const double* W_host,
                          itn_mpo** mpo) {
  if (!h || !mpo || !W_host) return h ? fail(h, ITN_E_ARG, "null argument") : ITN_E_ARG;
  *mpo = nullptr;
  if (N < 2 || w < 1 || d < 1) return fail(h, ITN_E_ARG, "need N >= 2, w >= 1, d >= 1");
  auto* o = new itn_mpo();
  o->N = N;
  o->w = w;
  o->d = d;
  o->W.assign(W_host, W_host + (size_t)N * w * w * d * d);
  *mpo = o;
  return ITN_OK;
}

itn_status itn_mpo_destroy(itn_mpo* mpo) {
  delete mpo;
  return ITN_OK;
}

itn_status itn_mps_create(itn_handle* h, int32_t N, int32_t d, const int32_t* bond,
                          const double* sites_host, itn_mps** mps) {
  if (!h || !mps || !bond || !sites_host) return h ? fail(h, ITN_E_ARG, "null argument") : ITN_E_ARG;
  *mps = nullptr;
  if (N < 2 || d < 1) return fail(h, ITN_E_ARG, "need N >= 2, d >= 1");
  if (bond[0] != 1 || bond[N] != 1) return fail(h, ITN_E_SHAPE, "bond[0] and bond[N] must be 1");
  for (int i = 0; i <= N; ++i)
    if (bond[i] < 1) return fail(h, ITN_E_SHAPE, "bond dimensions must be >= 1");
  if (h->device < 0) return fail(h, ITN_E_NODEVICE, "host-only handle cannot hold an MPS");
  auto* m = new itn_mps();
  m->N = N;
  m->d = d;
  m->bond.assign(bond, bond + N + 1);
  m->site.resize(N);
  m->Lenv.resize(N + 1);
  m->Renv.resize(N + 1);
  size_t off = 0;
  for (int i = 0; i < N; ++i) {
    const size_t n = (size_t)bond[i] * d * bond[i + 1];
    itn_status st = m->site[i].ensure(h, n * 8);
    if (st == ITN_OK && hipMemcpy(m->site[i].p, sites_host + off, n * 8, hipMemcpyHostToDevice) != hipSuccess)
      st = fail(h, ITN_E_HIP, "upload of site %d failed", i);
    if (st != ITN_OK) {
      delete m;
      return st;
    }
    off += n;
  }
  *mps = m;
  return ITN_OK;
}

itn_status itn_mps_destroy(itn_mps* mps) {
  if (mps) (void)hipDeviceSynchronize();
  delete mps;
  return ITN_OK;
}

itn_status itn_mps_bonds(const itn_mps* mps, int32_t* bond) {
  if (!mps || !bond) return ITN_E_ARG;
  std::copy(mps->bond.begin(), mps->bond.end(), bond);
  return ITN_OK;
}

itn_status itn_mps_get_site(itn_handle* h, const itn_mps* mps, int32_t i, double* host) {
  if (!h || !mps || !host) return ITN_E_ARG;
  if (i < 0 || i >= mps->N) return fail(h, ITN_E_ARG, "site index out of range");
  const size_t n = (size_t)mps->bond[i] * mps->d * mps->bond[i + 1];
  ITN_HIP(h, hipDeviceSynchronize());
  ITN_HIP(h, hipMemcpy(host, mps->site[i].p, n * 8, hipMemcpyDeviceToHost));
  return ITN_OK;
}

itn_status itn_dmrg_sweep(itn_handle* h, itn_mps* mps, const itn_mpo* mpo,
                          const itn_sweep_params* p, itn_sweep_result* res) {
  if (!h || !mps || !mpo || !p) return h ? fail(h, ITN_E_ARG, "null argument") : ITN_E_ARG;
  if (mpo->N != mps->N || mpo->d != mps->d)
    return fail(h, ITN_E_SHAPE, "MPO (N=%d, d=%d) does not match the MPS (N=%d, d=%d)", mpo->N,
                mpo->d, mps->N, mps->d);
  if (p->nsweeps < 0 || (p->nsweeps > 0 && (!p->maxdim || !p->cutoff)))
    return fail(h, ITN_E_ARG, "bad sweep schedule");
  if (p->prec != ITN_P_F64 && p->prec != ITN_P_F32 && p->prec != ITN_P_BF16)
    return fail(h, ITN_E_ARG, "unknown precision");
  for (int k = 0; k < p->nsweeps; ++k)
    if (p->maxdim[k] < 1 || p->cutoff[k] < 0) return fail(h, ITN_E_ARG, "bad maxdim/cutoff");
  if (h->device < 0) return fail(h, ITN_E_NODEVICE, "host-only handle cannot run sweeps");
  Ctx c;
  c.h = h;
  c.m = mps;
  c.mpo = mpo;
  c.p = p;
  const int N = mps->N;
  if (!mps->envs || mps->mpo_w != mpo->w) {
    ITN_TRY(boundary(c, mps->Lenv[0], mpo->w - 1));
    ITN_TRY(boundary(c, mps->Renv[N], 0));
    for (int i = N - 1; i >= 2; --i) ITN_TRY(env_step(c, i, false));
    mps->envs = true;
    mps->mpo_w = mpo->w;
  }
  if (p->northo < 0 || (p->northo > 0 && !p->ortho))
    return fail(h, ITN_E_ARG, "northo > 0 needs the ortho array");
  c.northo = p->northo;
  if (c.northo > 0) {
    for (int j = 0; j < c.northo; ++j) {
      const itn_mps* o = p->ortho[j];
      if (!o || o == mps) return fail(h, ITN_E_ARG, "ortho[%d] must be another MPS", j);
      if (o->N != N || o->d != mps->d)
        return fail(h, ITN_E_SHAPE, "ortho[%d] (N=%d, d=%d) does not match the MPS", j, o->N, o->d);
    }
    for (auto* v : {&mps->OL, &mps->OR}) {
      for (auto& row : *v)
        for (auto& b : row) b.release();
      v->assign(c.northo, std::vector<DBuf>(N + 1));
    }
    const double one = 1.0;
    for (int j = 0; j < c.northo; ++j) {
      const itn_mps* o = p->ortho[j];
      ITN_TRY(mps->OL[j][0].ensure(h, 8));
      ITN_TRY(mps->OR[j][N].ensure(h, 8));
      ITN_HIP(h, hipMemcpy(mps->OL[j][0].p, &one, 8, hipMemcpyHostToDevice));
      ITN_HIP(h, hipMemcpy(mps->OR[j][N].p, &one, 8, hipMemcpyHostToDevice));
      for (int k = N - 1; k >= 1; --k) {
        ITN_TRY(mps->OR[j][k].ensure(h, (size_t)mps->bond[k] * o->bond[k] * 8));
        ITN_TRY(ov_right(c, mps->OR[j][k + 1].d(), mps->site[k].d(), o->site[k].d(), mps->bond[k],
                         mps->bond[k + 1], o->bond[k], o->bond[k + 1], mps->OR[j][k].d()));
      }
    }
  }
  if (res) res->sweeps_done = 0;
  double prevE = 0.0;
  for (int sw = 0; sw < p->nsweeps; ++sw) {
    auto t0 = std::chrono::steady_clock::now();
    c.matvecs = 0;
    c.max_resid = 0.0;
    c.t_mv = c.t_solve = c.t_split = c.t_env = 0.0;
    double E = 0.0, maxtr = 0.0, tr = 0.0;
    for (int i = 0; i <= N - 2; ++i) {
      ITN_TRY(bond_step(c, i, true, p->maxdim[sw], p->cutoff[sw], &E, &tr));
      maxtr = std::max(maxtr, tr);
    }
    for (int i = N - 2; i >= 0; --i) {
      ITN_TRY(bond_step(c, i, false, p->maxdim[sw], p->cutoff[sw], &E, &tr));
      maxtr = std::max(maxtr, tr);
    }
    ITN_HIP(h, hipStreamSynchronize(c.s));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (res) {
      if (res->energy) res->energy[sw] = E;
      if (res->max_trunc) res->max_trunc[sw] = maxtr;
      if (res->max_bond) res->max_bond[sw] = *std::max_element(mps->bond.begin(), mps->bond.end());
      if (res->seconds) res->seconds[sw] = secs;
      if (res->matvecs) res->matvecs[sw] = c.matvecs;
      if (res->residual) res->residual[sw] = c.max_resid;
      if (p->timing) {
        if (res->t_matvec) res->t_matvec[sw] = c.t_mv;
        if (res->t_solver) res->t_solver[sw] = c.t_solve - c.t_mv;
        if (res->t_split) res->t_split[sw] = c.t_split;
        if (res->t_env) res->t_env[sw] = c.t_env;
      }
      res->sweeps_done = sw + 1;
    }
    if (sw > 0 && p->energy_tol > 0 && std::fabs(E - prevE) < p->energy_tol * std::fabs(E)) break;
    prevE = E;
  }
  if (c.unconverged)
    return fail(h, ITN_E_NOT_CONVERGED, "a local eigensolve ended above its tolerance (max residual %.3e)",
                c.max_resid);
  return ITN_OK;
}

}  // extern "C"
