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
#include <functional>

#include "common.h"
#include "dmrg_common.h"
#include "handle.h"

using namespace itn;


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
  SolverBufs sb;  // eigensolver scratch
  DBuf psi, tmp, rho, evec, eval, einfo, Lp, Rp, ev_host_stage;
  DBuf ovec, ot1, ot2, ot3, odots;
  DBuf hh, hscr;  // bond split: Householder reflectors [n][n]; tridiagonal and barrier scratch
  DBuf hdiag, wdiag;  // block Davidson: diagonal of H_eff, and its W1 W2 factor
  ~itn_mps() {
    for (auto& b : site) b.release();
    for (auto& b : Lenv) b.release();
    for (auto& b : Renv) b.release();
    for (auto* v : {&OL, &OR})
      for (auto& row : *v)
        for (auto& b : row) b.release();
    for (DBuf* b : {&psi, &tmp, &rho, &evec, &eval, &einfo, &Lp, &Rp, &ev_host_stage, &ovec, &ot1,
                    &ot2, &ot3, &odots, &hh, &hscr, &hdiag, &wdiag})
      b->release();
    sb.release();
  }
};

extern "C" void itn_release_solver(itn_handle* h) {
  if (h && h->solver) {
    rocblas_destroy_handle(static_cast<rocblas_handle>(h->solver));
    h->solver = nullptr;
  }
}

namespace itn {

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

}  // namespace itn

namespace {

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

struct Ctx : SolveCtx {
  itn_mps* m = nullptr;
  const itn_mpo* mpo = nullptr;
  // excited states: projected previous states at the current bond
  int northo = 0;
  const double* pen_v = nullptr;  // northo vectors of the bond's length
};

// y = H_eff x for nv vectors stored one after another (FP64), at precision
// `prec`, through the public entry point: one launch sequence for all nv.
itn_status heff(Ctx& c, int i, int prec, const double* x, double* y, int64_t cl, int64_t cr,
                int nv = 1) {
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
  ITN_TRY(itn_heff_apply(c.h, &L, &W1, &W2, &R, &P, nv, &O, (itn_prec)prec, c.s));
  if (c.northo > 0) {  // + weight * sum_j |v_j><v_j| x  (Sec. 7.2 energy penalty)
    const int64_t n = cl * d * d * cr;
    ITN_TRY(c.sb->partial.ensure(c.h, (size_t)c.northo * dot_blocks(n) * 8));
    ITN_TRY(c.m->odots.ensure(c.h, (size_t)c.northo * 8 + 8));
    for (int v = 0; v < nv; ++v) {
      ITN_HIP(c.h, multi_dot(c.pen_v, n, c.northo, x + (size_t)v * n, n, c.sb->partial.d(),
                             c.m->odots.d(), c.s));
      ITN_HIP(c.h, lincomb_dev(c.pen_v, n, c.northo, c.m->odots.d(), c.p->weight, y + (size_t)v * n,
                               n, c.s));
    }
  }
  return ITN_OK;
}

}  // namespace

namespace itn {

// Dot products of groups of vectors, read back with one host round trip:
// each add(V, k, w) queues <V_a, w> for a < k (V_a at stride n) into the
// next k slots of the result.
struct DotBatch {
  SolveCtx& c;
  int64_t n;
  int total = 0;
  std::vector<std::pair<int, int>> spans;  // (offset, count) per add
  DotBatch(SolveCtx& ctx, int64_t len) : c(ctx), n(len) {}
  itn_status add(const double* V, int k, const double* w, int* off) {
    ITN_TRY(c.sb->partial.ensure(c.h, (size_t)std::max(k, 1) * dot_blocks(n) * 8));
    ITN_TRY(c.sb->dots.ensure(c.h, (size_t)(total + k) * 8 + 8));
    ITN_HIP(c.h, multi_dot(V, n, k, w, n, c.sb->partial.d(), c.sb->dots.d() + total, c.s));
    *off = total;
    total += k;
    return ITN_OK;
  }
  itn_status read(std::vector<double>& out) {
    out.assign(std::max(total, 1), 0.0);
    if (total == 0) return ITN_OK;
    ITN_TRY(c.sb->pin.ensure(c.h, (size_t)total * 8 + 8));
    ITN_HIP(c.h, hipMemcpyAsync(c.sb->pin.p, c.sb->dots.p, (size_t)total * 8, hipMemcpyDeviceToHost, c.s));
    ITN_HIP(c.h, hipStreamSynchronize(c.s));
    std::memcpy(out.data(), c.sb->pin.p, (size_t)total * 8);
    return ITN_OK;
  }
};

// Lowest eigenpair of H_eff at bond i by Davidson (full
// re-orthogonalisation, restarts), FP64 basis.  psi (in/out, length n) is the
// start vector and the result.
//
// One vector per step (params->block <= 1): the residual of the lowest Ritz
// pair with the identity preconditioner (Lanczos-equivalent).  Host round
// trips per step: the residual's projections and norm, the new column of
// the projected matrix, and a second Gram-Schmidt pass only when the first
// removed more than half the residual's norm (Daniel-Gragg-Kaufman-Stewart).
//
// Block (params->block = B > 1): each step adds the residuals of the B
// lowest Ritz pairs, preconditioned with the diagonal of H_eff (Davidson's
// original correction (D - theta)^-1 r; with the identity all residuals of
// one Krylov space would be parallel), orthonormalised against the basis
// and each other by two rounds of Cholesky QR, and applies H_eff to the
// block in one batched launch (nv = accepted vectors, contiguous slots).
//
// Precision: matvecs of expansion vectors run at `prec`.  When prec is below
// FP64 and refinement is on, the vectors every restart cycle starts from
// (the start vector, then each restart's Ritz vectors) are applied in FP64
// instead: their rows and columns of the projected matrix are then exact,
// so the corrections found with low-precision matvecs enter the Ritz
// vectors with first-order-exact couplings and the iteration converges to
// the FP64 eigenpair (the low-precision error enters only through the
// corrections' own block, second order in their size).  A restart keeps one
// Ritz vector (with a block, the B lowest, all applied in FP64: with only
// the first exact, the others' low-precision couplings, of order u_bf16
// times the norm of H_eff, left Ritz vectors with residuals of that size),
// so a cycle is one (B) FP64 matvecs and the rest low-precision ones.  Without refinement every matvec runs at
// `prec`.  The returned energy is the Ritz value; with `exact_final` (mixed
// mode) a residual test passed with low-precision products is confirmed
// from a restart (FP64 products, then the exact residual), and a result
// that does not end on such a restart is applied once more in FP64: the
// returned energy and residual are then FP64 figures.
//
// *converged is false only when maxiter matvecs ended above the tolerance;
// a residual with no new direction left (the basis spans the invariant
// subspace up to rounding) counts as converged.
itn_status davidson(SolveCtx& c, const Matvec& mv, int prec, double tol, int maxiter, double* psi,
                    int64_t n, const double* diag, bool exact_final, double* energy, double* resid,
                    bool* converged) {
  // every H_eff application of the solve: counted, and timed as the matvec phase
  auto heff = [&](int p, const double* x, double* y, int nv) -> itn_status {
    PhaseTimer pt(c, &c.t_mv);
    c.matvecs += nv;
    if (p == ITN_P_F64) c.matvecs64 += nv;
    return mv(p, x, y, nv);
  };
  const bool mixed = prec != ITN_P_F64 && c.p->refine;
  const int B = diag ? std::max(1, std::min(c.p->block > 0 ? c.p->block : 1, 8)) : 1;
  const int keep_base = mixed ? 1 : 3;  // Ritz vectors kept at a restart
  int kmax = std::max(4, std::min(c.p->krylovdim, 32));
  kmax = std::max(kmax, std::max(keep_base, B) + B);
  // slots: basis [0, kmax), staged block [kmax, kmax + B), orthonormalisation
  // staging [kmax + B, kmax + 2B), restart staging, one spare
  const int s_orth = kmax + B, s_rest = kmax + 2 * B, s_spare = s_rest + std::max(keep_base, B);
  const int cap = s_spare + 1;
  ITN_TRY(c.sb->V.ensure(c.h, (size_t)cap * n * 8));
  ITN_TRY(c.sb->AV.ensure(c.h, (size_t)cap * n * 8));
  double* V = c.sb->V.d();
  double* AV = c.sb->AV.d();
  auto Vs = [&](int a) { return V + (size_t)a * n; };
  auto AVs = [&](int a) { return AV + (size_t)a * n; };
  std::vector<double> Hk((size_t)kmax * kmax, 0.0), got;
  auto H = [&](int a, int b) -> double& { return Hk[(size_t)a * kmax + b]; };
  int used = 0;  // matvecs of this solve
  {
    DotBatch db(c, n);
    int o;
    ITN_TRY(db.add(psi, 1, psi, &o));
    ITN_TRY(db.read(got));
  }
  const double nrm2 = got[0];
  if (!(nrm2 > 0)) return fail(c.h, ITN_E_ARG, "zero start vector");
  ITN_HIP(c.h, hipMemcpyAsync(V, psi, n * 8, hipMemcpyDeviceToDevice, c.s));
  ITN_HIP(c.h, scale(V, 1.0 / std::sqrt(nrm2), n, c.s));
  ITN_TRY(heff(mixed ? ITN_P_F64 : prec, V, AV, 1));
  ++used;
  {
    DotBatch db(c, n);
    int o;
    ITN_TRY(db.add(V, 1, AV, &o));
    ITN_TRY(db.read(got));
    H(0, 0) = got[0];
  }
  int k = 1;
  int nexact = 1;  // leading basis vectors whose products are FP64 (mixed mode)
  double theta = H(0, 0), rn = 0.0;
  bool conv = false, force_restart = false;
  std::vector<double> w, Y, y0(1, 1.0);
  // Orthonormalise the nin vectors in slots [k, k + nin) against the basis
  // and each other, from their projections P(j, a) = <V_a, t_j> (a < k) and
  // Gram matrix P(j, k + l): subtract the projections, Cholesky of the
  // block's Gram (directions whose pivot is below drop * ref[j] are left out),
  // accepted vectors written back to [k, k + *nout).
  auto cholqr = [&](int nin, const std::function<double(int, int)>& P, double drop,
                    const std::vector<double>& ref, int* nout) -> itn_status {
    for (int j = 0; j < nin; ++j) {
      std::vector<double> cj(k);
      for (int a = 0; a < k; ++a) cj[a] = -P(j, a);
      ITN_HIP(c.h, lincomb(V, n, k, cj.data(), 1.0, Vs(k + j), n, c.s));
    }
    std::vector<double> Gb((size_t)nin * nin), Lc((size_t)nin * nin, 0.0);
    for (int j = 0; j < nin; ++j)
      for (int l = 0; l < nin; ++l) {
        double v = P(j, k + l);
        for (int a = 0; a < k; ++a) v -= P(j, a) * P(l, a);
        Gb[(size_t)j * nin + l] = v;
      }
    std::vector<int> idx;
    for (int j = 0; j < nin; ++j) {
      double piv = Gb[(size_t)j * nin + j];
      for (int q : idx) piv -= Lc[(size_t)j * nin + q] * Lc[(size_t)j * nin + q];
      if (!(piv > drop * ref[j])) continue;
      const double lj = std::sqrt(piv);
      Lc[(size_t)j * nin + j] = lj;
      for (int l = j + 1; l < nin; ++l) {
        double v = Gb[(size_t)l * nin + j];
        for (int q : idx) v -= Lc[(size_t)l * nin + q] * Lc[(size_t)j * nin + q];
        Lc[(size_t)l * nin + j] = v / lj;
      }
      idx.push_back(j);
    }
    const int na = (int)idx.size();
    // t_q = sum_j T[q][j] r_j: forward substitution over the accepted columns
    std::vector<double> T((size_t)std::max(na, 1) * nin, 0.0);
    for (int q = 0; q < na; ++q) {
      const int j = idx[q];
      std::vector<double> cf(nin, 0.0);
      cf[j] = 1.0;
      for (int p = 0; p < q; ++p) {
        const double lij = Lc[(size_t)j * nin + idx[p]];
        for (int jj = 0; jj < nin; ++jj) cf[jj] -= lij * T[(size_t)p * nin + jj];
      }
      for (int jj = 0; jj < nin; ++jj) T[(size_t)q * nin + jj] = cf[jj] / Lc[(size_t)j * nin + j];
    }
    for (int q = 0; q < na; ++q)
      ITN_HIP(c.h, lincomb(Vs(k), n, nin, &T[(size_t)q * nin], 0.0, Vs(s_orth + q), n, c.s));
    if (na > 0)
      ITN_HIP(c.h, hipMemcpyAsync(Vs(k), Vs(s_orth), (size_t)na * n * 8, hipMemcpyDeviceToDevice, c.s));
    *nout = na;
    return ITN_OK;
  };
  for (;;) {
    // Ritz pairs of the projected problem
    std::vector<double> Hs((size_t)k * k);
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b) Hs[a * k + b] = 0.5 * (H(a, b) + H(b, a));
    jacobi_eigh(k, Hs, w, Y);
    theta = w[0];
    y0.assign(k, 0.0);
    for (int a = 0; a < k; ++a) y0[a] = Y[a * k + 0];
    const int nb = std::min(B, k);
    // residuals of the nb lowest pairs, staged in slots k .. k+nb-1
    for (int j = 0; j < nb; ++j) {
      std::vector<double> yj(k), ny(k);
      for (int a = 0; a < k; ++a) {
        yj[a] = Y[a * k + j];
        ny[a] = -w[j] * yj[a];
      }
      ITN_HIP(c.h, lincomb(AV, n, k, yj.data(), 0.0, Vs(k + j), n, c.s));
      ITN_HIP(c.h, lincomb(V, n, k, ny.data(), 1.0, Vs(k + j), n, c.s));
    }
    if (B > 1) {  // keep the lowest pair's residual for the convergence test, precondition all
      ITN_HIP(c.h, hipMemcpyAsync(Vs(s_spare), Vs(k), n * 8, hipMemcpyDeviceToDevice, c.s));
      for (int j = 0; j < nb; ++j)
        ITN_HIP(c.h, precond_diag(Vs(k + j), diag, w[j], 1e-2 * std::max(1.0, std::fabs(w[j])), n, c.s));
    }
    // projections on the basis and the block's Gram matrix: G(j, a) = <V_a, t_j>, a < k + nb
    std::vector<int> off(nb);
    int orr = 0;
    {
      DotBatch db(c, n);
      for (int j = 0; j < nb; ++j) ITN_TRY(db.add(V, k + nb, Vs(k + j), &off[j]));
      if (B > 1) ITN_TRY(db.add(Vs(s_spare), 1, Vs(s_spare), &orr));
      ITN_TRY(db.read(got));
    }
    std::vector<double> G0 = got;
    auto G = [&](int j, int a) { return G0[off[j] + a]; };
    rn = std::sqrt(std::max(B > 1 ? G0[orr] : G(0, k), 0.0));
    if (rn <= tol * std::max(1.0, std::fabs(theta))) {
      // In mixed mode a residual formed from low-precision products (k > 1)
      // can pass the test while the FP64 residual does not.  Where the
      // result must hold in FP64 (exact_final), confirm it from a restart:
      // its single vector's product is FP64, so the next residual is exact.
      if (!(mixed && exact_final && k > nexact && used < maxiter)) {
        conv = true;
        break;
      }
      force_restart = true;
    }
    if (used >= maxiter) break;
    if (k + nb > kmax || force_restart) {
      force_restart = false;
      // restart from the m lowest Ritz vectors (staged, then moved to the front)
      const int m = std::min(k, std::max(keep_base, nb));
      for (int j = 0; j < m; ++j) {
        std::vector<double> yj(k);
        for (int a = 0; a < k; ++a) yj[a] = Y[a * k + j];
        ITN_HIP(c.h, lincomb(V, n, k, yj.data(), 0.0, Vs(s_rest + j), n, c.s));
        ITN_HIP(c.h, lincomb(AV, n, k, yj.data(), 0.0, AVs(s_rest + j), n, c.s));
      }
      ITN_HIP(c.h, hipMemcpyAsync(V, Vs(s_rest), (size_t)m * n * 8, hipMemcpyDeviceToDevice, c.s));
      ITN_HIP(c.h, hipMemcpyAsync(AV, AVs(s_rest), (size_t)m * n * 8, hipMemcpyDeviceToDevice, c.s));
      std::fill(Hk.begin(), Hk.end(), 0.0);
      for (int j = 0; j < m; ++j) H(j, j) = w[j];
      k = m;
      if (mixed) {  // the kept vectors applied in FP64: their rows and columns are exact
        ITN_TRY(heff(ITN_P_F64, V, AV, m));
        used += m;
        DotBatch db(c, n);
        std::vector<int> o(m);
        for (int b = 0; b < m; ++b) ITN_TRY(db.add(V, m, AVs(b), &o[b]));
        ITN_TRY(db.read(got));
        for (int b = 0; b < m; ++b)
          for (int a = 0; a <= b; ++a)
            H(a, b) = H(b, a) = 0.5 * (got[o[b] + a] + got[o[a] + b]);
        nexact = m;
      }
      continue;
    }
    const int nbb = std::min(nb, maxiter - used);
    int na = 0;
    if (B == 1) {
      // one residual: classical Gram-Schmidt, a second pass when the first
      // removed more than half of its norm; no new direction left when the
      // second pass keeps less than 1e-28 of it
      const double r2 = G(0, k);
      std::vector<double> ref(1, r2);
      double t2 = r2;
      for (int a = 0; a < k; ++a) t2 -= G(0, a) * G(0, a);
      if (!(t2 > 0.5 * r2)) {
        std::vector<double> cj(k);
        for (int a = 0; a < k; ++a) cj[a] = -G(0, a);
        ITN_HIP(c.h, lincomb(V, n, k, cj.data(), 1.0, Vs(k), n, c.s));
        DotBatch db(c, n);
        int o;
        ITN_TRY(db.add(V, k + 1, Vs(k), &o));
        ITN_TRY(db.read(got));
        std::vector<double> G1(got.begin() + o, got.begin() + o + k + 1);
        ITN_TRY(cholqr(1, [&](int, int a) { return G1[a]; }, 1e-28, ref, &na));
      } else {
        ITN_TRY(cholqr(1, [&](int j, int a) { return G(j, a); }, 1e-28, ref, &na));
      }
    } else {
      // a block: two rounds of Cholesky QR (the second from fresh products,
      // on vectors already close to orthonormal)
      std::vector<double> ref(nbb);
      for (int j = 0; j < nbb; ++j) ref[j] = G(j, k + j);
      ITN_TRY(cholqr(nbb, [&](int j, int a) { return G(j, a); }, 1e-20, ref, &na));
      if (na > 0) {
        std::vector<int> o2(na);
        DotBatch db(c, n);
        for (int q = 0; q < na; ++q) ITN_TRY(db.add(V, k + na, Vs(k + q), &o2[q]));
        ITN_TRY(db.read(got));
        std::vector<double> G2 = got, ones(na, 1.0);
        const int na1 = na;
        ITN_TRY(cholqr(na1, [&](int j, int a) { return G2[o2[j] + a]; }, 1e-10, ones, &na));
      }
    }
    if (na == 0) {
      // the basis holds the invariant subspace up to rounding.  In mixed
      // precision the residual above was formed with low-precision products:
      // restart from the Ritz vector (its FP64 product makes the next
      // residual exact) unless the basis is that single vector already.
      if (mixed && k > 1) {
        force_restart = true;
        continue;
      }
      conv = true;
      break;
    }
    // one batched matvec for the accepted vectors
    ITN_TRY(heff(prec, Vs(k), AVs(k), na));
    used += na;
    // new columns of the projected matrix; in mixed mode row 0 from the exact AV_0
    {
      DotBatch db(c, n);
      std::vector<int> oc(na), o0(na);
      for (int q = 0; q < na; ++q) ITN_TRY(db.add(V, k + na, AVs(k + q), &oc[q]));
      if (mixed)
        for (int q = 0; q < na; ++q) ITN_TRY(db.add(AV, nexact, Vs(k + q), &o0[q]));
      ITN_TRY(db.read(got));
      for (int q = 0; q < na; ++q)
        for (int a = 0; a <= k + q; ++a) H(a, k + q) = H(k + q, a) = got[oc[q] + a];
      for (int q = 0; q < na; ++q)
        for (int l = q + 1; l < na; ++l)  // symmetric average inside the block
          H(k + q, k + l) = H(k + l, k + q) = 0.5 * (got[oc[l] + k + q] + got[oc[q] + k + l]);
      if (mixed)
        for (int q = 0; q < na; ++q)
          for (int a = 0; a < nexact; ++a) H(a, k + q) = H(k + q, a) = got[o0[q] + a];
    }
    k += na;
  }
  // the Ritz vector of the last projected problem
  ITN_HIP(c.h, lincomb(V, n, k, y0.data(), 0.0, psi, n, c.s));
  // A basis of only the vectors applied in FP64 (after a restart, or the
  // start) holds the FP64 products already: theta and rn are FP64 figures.
  const bool exact_now = mixed && k == nexact;
  if (mixed && exact_final && !exact_now) {
    // FP64 Rayleigh quotient and residual of the result
    double* ax = AVs(s_spare);
    ITN_TRY(heff(ITN_P_F64, psi, ax, 1));
    DotBatch db(c, n);
    int o1, o2;
    ITN_TRY(db.add(psi, 1, ax, &o1));
    ITN_TRY(db.add(psi, 1, psi, &o2));
    ITN_TRY(db.read(got));
    const double xx = got[o2];
    theta = got[o1] / xx;
    double* r = Vs(s_spare);
    const double cf[2] = {1.0, -theta};
    ITN_HIP(c.h, lincomb(ax, n, 1, cf, 0.0, r, n, c.s));
    ITN_HIP(c.h, lincomb(psi, n, 1, cf + 1, 1.0, r, n, c.s));
    DotBatch db2(c, n);
    ITN_TRY(db2.add(r, 1, r, &o1));
    ITN_TRY(db2.read(got));
    rn = std::sqrt(std::max(got[o1], 0.0) / xx);
    conv = rn <= tol * std::max(1.0, std::fabs(theta));
  }
  *energy = theta;
  *resid = rn;
  *converged = conv;
  return ITN_OK;
}

}  // namespace itn

namespace {

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
    ITN_TRY(m->sb.pin.ensure(c.h, (size_t)(n + 2) * 8));
    char* pin = static_cast<char*>(m->sb.pin.p);
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
    ITN_TRY(m->sb.pin.ensure(c.h, (size_t)(n + 2) * 8));
    char* pin = static_cast<char*>(m->sb.pin.p);
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
itn_status bond_step(Ctx& c, int i, bool to_right, int maxdim, double cutoff, bool last,
                     double* energy, double* trunc) {
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
  const double* diag = nullptr;
  if (c.p->block > 1) {  // the diagonal of H_eff for the block expansion's preconditioner
    const int w = c.mpo->w, d2 = d * d;
    std::vector<double> wd((size_t)w * w * d2, 0.0);
    const double* W1 = c.mpo->site(i);
    const double* W2 = c.mpo->site(i + 1);
    for (int m0 = 0; m0 < w; ++m0)
      for (int m2 = 0; m2 < w; ++m2)
        for (int s1 = 0; s1 < d; ++s1)
          for (int s2 = 0; s2 < d; ++s2) {
            double v = 0.0;
            for (int m1 = 0; m1 < w; ++m1)
              v += W1[((m0 * w + m1) * d + s1) * d + s1] * W2[((m1 * w + m2) * d + s2) * d + s2];
            wd[((size_t)m0 * w + m2) * d2 + s1 * d + s2] = v;
          }
    ITN_TRY(m->wdiag.ensure(c.h, wd.size() * 8));
    ITN_TRY(m->hdiag.ensure(c.h, (size_t)n * 8));
    ITN_HIP(c.h, hipMemcpyAsync(m->wdiag.p, wd.data(), wd.size() * 8, hipMemcpyHostToDevice, c.s));
    ITN_HIP(c.h, heff_diag(m->Lenv[i].d(), m->Renv[i + 2].d(), m->wdiag.d(), w, d2, cl, cr,
                           m->hdiag.d(), c.s));
    diag = m->hdiag.d();
  }
  {
    PhaseTimer pt(c, &c.t_solve);
    const Matvec mv = [&](int p, const double* x, double* y, int nv) {
      return heff(c, i, p, x, y, cl, cr, nv);
    };
    ITN_TRY(davidson(c, mv, prec, tol, maxiter, m->psi.d(), n, diag, last, &e, &r, &conv));
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
  c.sb = &mps->sb;
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
    c.matvecs64 = 0;
    c.max_resid = 0.0;
    c.t_mv = c.t_solve = c.t_split = c.t_env = 0.0;
    double E = 0.0, maxtr = 0.0, tr = 0.0;
    for (int i = 0; i <= N - 2; ++i) {
      ITN_TRY(bond_step(c, i, true, p->maxdim[sw], p->cutoff[sw], false, &E, &tr));
      maxtr = std::max(maxtr, tr);
    }
    for (int i = N - 2; i >= 0; --i) {
      ITN_TRY(bond_step(c, i, false, p->maxdim[sw], p->cutoff[sw], i == 0, &E, &tr));
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
      if (res->matvecs_f64) res->matvecs_f64[sw] = c.matvecs64;
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
