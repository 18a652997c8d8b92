// Block-sparse (quantum-number) two-site DMRG: the sweep of Sec. 7.2 with
// every tensor stored as QN blocks (Sec. 8, 9.2).  The local problem is the
// planned block-sparse H_eff (itn_qn_heff_plan / apply), the environments
// are three block-sparse contractions each (itn_contract), and the bond is
// split sector by sector: the two-site tensor is a block-diagonal matrix
// over the new link's charge, each charge sector's density matrix is
// diagonalised, and the truncation of Sec. 5 is applied to the weights of
// all sectors together.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <set>

#include "dmrg_common.h"
#include "handle.h"
#include "qn_common.h"

using namespace itn;
using namespace itn::qn;

namespace {

// A block-sparse tensor held by the library: structure, flux, FP64 data.
struct QBT {
  QTensor q;
  std::vector<int32_t> flux;
  DBuf data;
  double* d() const { return data.d(); }
};

// The ABI view of a QTensor (arrays kept alive with it); `flip` reverses
// every arrow (the conjugate tensor dag(T): real data, same blocks).
struct View {
  std::vector<std::vector<int32_t>> qn, dim, mod;
  std::vector<itn_space> sp;
  std::vector<int64_t> dims, boff;
  std::vector<int32_t> labels, bsec, flux;
  itn_tensor t{};
  View(const QTensor& q, const std::vector<int32_t>& fl, const void* data, itn_dtype dt,
       const std::vector<int32_t>& lab = {}, bool flip = false) {
    const int r = q.rank;
    qn.resize(r);
    dim.resize(r);
    mod.resize(r);
    sp.resize(r);
    for (int i = 0; i < r; ++i) {
      const QSpace& s = q.sp[i];
      qn[i] = s.qn;
      dim[i] = s.dim;
      mod[i] = s.mod;
      sp[i].nsec = s.nsec;
      sp[i].nq = s.nq;
      sp[i].qn = qn[i].data();
      sp[i].dim = dim[i].data();
      sp[i].arrow = flip ? (int8_t)-s.arrow : s.arrow;
      sp[i].mod = mod[i].data();
      dims.push_back(s.total);
    }
    for (auto& b : q.blocks) bsec.insert(bsec.end(), b.begin(), b.end());
    boff = q.off;
    labels = lab;
    flux = fl;
    if (flip && !flux.empty()) {
      const auto& m = q.sp[0].mod;
      for (size_t c = 0; c < flux.size(); ++c) flux[c] = qn_red(-(int64_t)flux[c], m[c]);
    }
    t.rank = r;
    t.dims = dims.data();
    t.label = labels.empty() ? nullptr : labels.data();
    t.space = sp.data();
    t.dtype = dt;
    t.data = const_cast<void*>(data);
    t.nblocks = (int64_t)q.blocks.size();
    t.block_sec = bsec.data();
    t.block_off = boff.data();
    t.flux = flux.empty() ? nullptr : flux.data();
  }
};

// A tensor structure from its indices and block list (offsets filled in).
QTensor make_qt(const std::vector<QSpace>& sp, const std::vector<std::vector<int32_t>>& blocks) {
  QTensor q;
  q.rank = (int)sp.size();
  q.sp = sp;
  int64_t o = 0;
  for (auto& b : blocks) {
    int64_t sz = 1;
    for (int i = 0; i < q.rank; ++i) sz *= q.sp[i].dim[b[i]];
    q.index[b] = (int)q.blocks.size();
    q.blocks.push_back(b);
    q.off.push_back(o);
    o += sz;
  }
  q.elems = o;
  return q;
}

QSpace with_arrow(QSpace s, int8_t a) {
  s.arrow = a;
  return s;
}

// QN index from the QNs of a basis (maximal runs of equal QN are sectors).
QSpace space_from_basis(const int32_t* qns, int n, int nq, const std::vector<int32_t>& mod, int8_t arrow) {
  QSpace s;
  s.nq = nq;
  s.mod = mod;
  s.arrow = arrow;
  for (int k = 0; k < n; ++k) {
    std::vector<int32_t> q(nq);
    for (int c = 0; c < nq; ++c) q[c] = qn_red(qns[k * nq + c], mod[c]);
    if (s.nsec > 0 && std::equal(q.begin(), q.end(), s.q(s.nsec - 1))) {
      s.dim.back()++;
    } else {
      s.qn.insert(s.qn.end(), q.begin(), q.end());
      s.dim.push_back(1);
      s.nsec++;
    }
  }
  s.off.resize(s.nsec);
  s.total = 0;
  for (int k = 0; k < s.nsec; ++k) {
    s.off[k] = s.total;
    s.total += s.dim[k];
  }
  return s;
}

QSpace single_sector(const std::vector<int32_t>& q, const std::vector<int32_t>& mod, int8_t arrow) {
  QSpace s;
  s.nq = (int)q.size();
  s.mod = mod;
  s.arrow = arrow;
  s.nsec = 1;
  s.qn = q;
  s.dim = {1};
  s.off = {0};
  s.total = 1;
  return s;
}

// sector and position of basis state k of a space built by space_from_basis
std::pair<int, int> locate(const QSpace& s, int k) {
  for (int j = 0; j < s.nsec; ++j)
    if (k < s.off[j] + s.dim[j]) return {j, (int)(k - s.off[j])};
  return {-1, -1};
}

}  // namespace

struct itn_qn_mps {
  int32_t N = 0, d = 0, nq = 0;
  std::vector<int32_t> mod;
  QSpace site;                  // physical index (arrow Out)
  std::vector<QSpace> link;     // N + 1 link indices (stored with arrow Out)
  std::vector<QBT> A;           // sites [a:Out, s:Out, a':In], flux 0
  std::vector<QBT> L, R;        // L[k] left of bond k [a':Out, m:In, a:In]; R[k] [b':In, m:Out, b:Out]
  bool envs = false;
  std::vector<int32_t> env_link_qn;  // MPO channel QNs the environments were built with
  const itn_mpo* env_mpo = nullptr;
  SolverBufs sb;
  DBuf psi, Lp, Rp, mat, matT, rho, ut, prod, ev, info, bat, batw, bmeta;
  DBuf hdiag, dtab, bx, by;  // block Davidson: H_eff diagonal, its tables, padded batches
  DBuf ctab[4];                    // bond split: tables of its batched copies
  QBT theta, T1, T2;  // two-site tensor and environment intermediates (buffers reused)
  HostPin pin;
  ~itn_qn_mps() {
    for (auto* v : {&A, &L, &R})
      for (auto& t : *v) t.data.release();
    for (QBT* t : {&theta, &T1, &T2}) t->data.release();
    for (DBuf& b : ctab) b.release();
    for (DBuf* b : {&psi, &Lp, &Rp, &mat, &matT, &rho, &ut, &prod, &ev, &info, &bat, &batw, &bmeta,
                    &hdiag, &dtab, &bx, &by})
      b->release();
    sb.release();
    pin.release();
  }
};

namespace itn {
namespace qn {

itn_status heff_diag_build(itn_handle* h, const QTensor& L, const QTensor& R, const double* W1,
                           const double* W2, int wm, const QTensor& P, HeffDiag& out) {
  if (!P.sp[0].same_sectors(L.sp[0]) || !P.sp[3].same_sectors(R.sp[0]))
    return fail(h, ITN_E_SHAPE, "the environments' link sectors differ from psi's");
  const QSpace &ML = L.sp[1], &MR = R.sp[1];
  const int wl = (int)ML.total, wr = (int)MR.total, d1 = (int)P.sp[1].total, d2 = (int)P.sp[2].total;
  // zero-charge channels of each environment (only these reach the diagonal)
  auto zeros = [](const QSpace& sp, std::vector<int32_t>& zpos) {
    zpos.assign((size_t)sp.total, -1);
    int n = 0;
    for (int k = 0; k < sp.nsec; ++k) {
      bool zero = true;
      for (int c = 0; c < sp.nq; ++c) zero &= qn_red(sp.q(k)[c], sp.mod[c]) == 0;
      if (zero)
        for (int y = 0; y < sp.dim[k]; ++y) zpos[(size_t)(sp.off[k] + y)] = n++;
    }
    return std::max(n, 1);
  };
  std::vector<int32_t> zl, zr;
  out.wzl = zeros(ML, zl);
  out.wzr = zeros(MR, zr);
  out.d1 = d1;
  out.d2 = d2;
  std::vector<double> wd((size_t)out.wzl * out.wzr * d1 * d2, 0.0);
  for (int m0 = 0; m0 < wl; ++m0)
    for (int m2 = 0; m2 < wr; ++m2) {
      if (zl[(size_t)m0] < 0 || zr[(size_t)m2] < 0) continue;
      for (int s1 = 0; s1 < d1; ++s1)
        for (int s2 = 0; s2 < d2; ++s2) {
          double v = 0.0;
          for (int m1 = 0; m1 < wm; ++m1)
            v += W1[(((size_t)m0 * wm + m1) * d1 + s1) * d1 + s1] *
                 W2[(((size_t)m1 * wr + m2) * d2 + s2) * d2 + s2];
          wd[(((size_t)zl[(size_t)m0] * out.wzr + zr[(size_t)m2]) * d1 + s1) * d2 + s2] = v;
        }
    }
  auto items = [&](const QTensor& E, const std::vector<int32_t>& zpos,
                   std::vector<EnvDiagItem>& v) -> itn_status {
    for (size_t b = 0; b < E.blocks.size(); ++b) {
      const auto& k = E.blocks[b];
      if (k[0] != k[2]) continue;
      const int64_t mg = E.sp[1].off[k[1]];
      if (zpos[(size_t)mg] < 0)
        return fail(h, ITN_E_FLUX, "environment block with equal link sectors on a charged channel");
      v.push_back({E.off[b], E.sp[0].dim[k[0]], E.sp[1].dim[k[1]], E.sp[0].off[k[0]], zpos[(size_t)mg]});
    }
    return ITN_OK;
  };
  std::vector<EnvDiagItem> li, ri;
  ITN_TRY(items(L, zl, li));
  ITN_TRY(items(R, zr, ri));
  std::vector<DiagBlock> db;
  out.most = 0;
  for (size_t b = 0; b < P.blocks.size(); ++b) {
    const auto& k = P.blocks[b];
    DiagBlock q{P.off[b],          P.sp[0].dim[k[0]], P.sp[1].dim[k[1]], P.sp[2].dim[k[2]], P.sp[3].dim[k[3]],
                P.sp[0].off[k[0]], P.sp[1].off[k[1]], P.sp[2].off[k[2]], P.sp[3].off[k[3]]};
    out.most = std::max(out.most, q.da * q.d1 * q.d2 * q.db);
    db.push_back(q);
  }
  out.cl = P.sp[0].total;
  out.cr = P.sp[3].total;
  out.nli = (int)li.size();
  out.nri = (int)ri.size();
  out.ndb = (int)db.size();
  out.o_li = wd.size() * 8;
  out.o_ri = out.o_li + li.size() * sizeof(EnvDiagItem);
  out.o_db = out.o_ri + ri.size() * sizeof(EnvDiagItem);
  out.host.assign(out.o_db + db.size() * sizeof(DiagBlock), 0);
  std::memcpy(out.host.data(), wd.data(), wd.size() * 8);
  if (!li.empty()) std::memcpy(out.host.data() + out.o_li, li.data(), li.size() * sizeof(EnvDiagItem));
  if (!ri.empty()) std::memcpy(out.host.data() + out.o_ri, ri.data(), ri.size() * sizeof(EnvDiagItem));
  if (!db.empty()) std::memcpy(out.host.data() + out.o_db, db.data(), db.size() * sizeof(DiagBlock));
  return ITN_OK;
}

hipError_t heff_diag_launch(const HeffDiag& q, const double* Ldata, const double* Rdata, void* dev, double* D,
                            hipStream_t s) {
  char* dt = static_cast<char*>(dev);
  double* Ld = reinterpret_cast<double*>(dt + round256(q.host.size()));
  double* Rd = Ld + (size_t)q.cl * q.wzl;
  hipError_t e = hipMemcpyAsync(dt, q.host.data(), q.host.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(Ld, 0, (size_t)(q.cl * q.wzl + q.cr * q.wzr) * 8, s);
  if (e == hipSuccess)
    e = env_diag_gather(Ldata, reinterpret_cast<const EnvDiagItem*>(dt + q.o_li), q.nli, q.wzl, Ld, s);
  if (e == hipSuccess)
    e = env_diag_gather(Rdata, reinterpret_cast<const EnvDiagItem*>(dt + q.o_ri), q.nri, q.wzr, Rd, s);
  if (e == hipSuccess)
    e = qn_heff_diag(Ld, Rd, reinterpret_cast<const double*>(dt), q.wzl, q.wzr, q.d1, q.d2,
                     reinterpret_cast<const DiagBlock*>(dt + q.o_db), q.ndb, (q.most + 255) / 256, D, s);
  return e;
}

}  // namespace qn
}  // namespace itn

namespace {

struct QCtx : SolveCtx {
  itn_qn_mps* m = nullptr;
  int sweep = 0;
  const itn_mpo* mpo = nullptr;
  QSpace mlink;                 // MPO link index (arrow Out)
  std::vector<QBT> W;           // MPO sites as block tensors (device), [m:Out, m':In, s':Out, s:In]
};

itn_status upload(itn_handle* h, QBT& t, const std::vector<double>& host) {
  ITN_TRY(t.data.ensure(h, std::max<size_t>(8, host.size() * 8)));
  if (!host.empty())
    ITN_HIP(h, hipMemcpy(t.data.p, host.data(), host.size() * 8, hipMemcpyHostToDevice));
  return ITN_OK;
}

// The block-sparse product C = A * B (labels as itn_contract), C's structure
// from A's and B's indices: every flux-allowed block when `all_blocks`,
// else the blocks reached by contributing pairs.  C's data is (re)sized.
itn_status contract(QCtx& c, const QBT& A, const std::vector<int32_t>& la, bool dagA, const QBT& B,
                    const std::vector<int32_t>& lb, bool dagB, const std::vector<int32_t>& lc, QBT& C,
                    bool all_blocks = false) {
  const auto& mod = c.m->mod;
  auto arrow_of = [](const QSpace& s, bool flip) { return (int8_t)(flip ? -s.arrow : s.arrow); };
  std::vector<QSpace> sp(lc.size());
  for (size_t k = 0; k < lc.size(); ++k) {
    bool found = false;
    for (int i = 0; i < A.q.rank && !found; ++i)
      if (la[i] == lc[k]) sp[k] = with_arrow(A.q.sp[i], arrow_of(A.q.sp[i], dagA)), found = true;
    for (int i = 0; i < B.q.rank && !found; ++i)
      if (lb[i] == lc[k]) sp[k] = with_arrow(B.q.sp[i], arrow_of(B.q.sp[i], dagB)), found = true;
    if (!found) return fail(c.h, ITN_E_LABEL, "internal: output label %d not found", lc[k]);
  }
  auto sgn = [](bool f) { return f ? -1 : 1; };
  std::vector<int32_t> fl(c.m->nq);
  for (int q = 0; q < c.m->nq; ++q)
    fl[q] = qn_red((int64_t)sgn(dagA) * A.flux[q] + (int64_t)sgn(dagB) * B.flux[q], mod[q]);
  std::vector<std::vector<int32_t>> blocks;
  if (all_blocks) {
    QTensor probe = make_qt(sp, {});
    blocks = allowed_blocks(probe, fl);
  } else {
    std::map<std::vector<int32_t>, std::vector<int>> bsec;
    std::vector<std::pair<int, int>> con;  // (axis in A, axis in B)
    for (int i = 0; i < A.q.rank; ++i)
      for (int j = 0; j < B.q.rank; ++j)
        if (la[i] == lb[j]) con.push_back({i, j});
    for (size_t b = 0; b < B.q.blocks.size(); ++b) {
      std::vector<int32_t> key;
      for (auto& p : con) key.push_back(B.q.blocks[b][p.second]);
      bsec[key].push_back((int)b);
    }
    std::set<std::vector<int32_t>> out;
    for (size_t a = 0; a < A.q.blocks.size(); ++a) {
      std::vector<int32_t> key;
      for (auto& p : con) key.push_back(A.q.blocks[a][p.first]);
      auto it = bsec.find(key);
      if (it == bsec.end()) continue;
      for (int b : it->second) {
        std::vector<int32_t> cb(lc.size());
        for (size_t k = 0; k < lc.size(); ++k) {
          for (int i = 0; i < A.q.rank; ++i)
            if (la[i] == lc[k]) cb[k] = A.q.blocks[a][i];
          for (int i = 0; i < B.q.rank; ++i)
            if (lb[i] == lc[k]) cb[k] = B.q.blocks[b][i];
        }
        out.insert(cb);
      }
    }
    blocks.assign(out.begin(), out.end());
  }
  C.q = make_qt(sp, blocks);
  C.flux = fl;
  ITN_TRY(C.data.ensure(c.h, std::max<int64_t>(C.q.elems, 1) * 8));
  View va(A.q, A.flux, A.d(), ITN_F64, la, dagA), vb(B.q, B.flux, B.d(), ITN_F64, lb, dagB),
      vc(C.q, C.flux, C.d(), ITN_F64, lc);
  return itn_contract(c.h, &va.t, &vb.t, &vc.t, ITN_P_F64, c.s);
}

// L_{i+1} from L_i and site i:  L'[a'', m', a'''] = sum L[a', m, a] A[a', s', a''] W[m, m', s', s] A[a, s, a''']
// R_i from R_{i+1} and site i:  R'[b', m, b] = sum A[b', s', b''] W[m, m', s', s] A[b, s, b'''] R[b'', m', b''']
itn_status env_step(QCtx& c, int i, bool left) {
  itn_qn_mps* m = c.m;
  QBT &T1 = m->T1, &T2 = m->T2;  // buffers kept between steps (stream order protects them)
  if (left) {
    ITN_TRY(contract(c, m->L[i], {1, 2, 3}, false, m->A[i], {1, 4, 5}, true, {2, 3, 4, 5}, T1));
    ITN_TRY(contract(c, T1, {2, 3, 4, 5}, false, c.W[i], {2, 6, 4, 7}, false, {3, 5, 6, 7}, T2));
    ITN_TRY(contract(c, T2, {3, 5, 6, 7}, false, m->A[i], {3, 7, 8}, false, {5, 6, 8}, m->L[i + 1]));
  } else {
    ITN_TRY(contract(c, m->A[i], {1, 4, 5}, true, m->R[i + 1], {5, 6, 7}, false, {1, 4, 6, 7}, T1));
    ITN_TRY(contract(c, T1, {1, 4, 6, 7}, false, c.W[i], {8, 6, 4, 9}, false, {1, 7, 8, 9}, T2));
    ITN_TRY(contract(c, T2, {1, 7, 8, 9}, false, m->A[i], {10, 9, 7}, false, {1, 8, 10}, m->R[i]));
  }
  return ITN_OK;
}

rocblas_handle solver(QCtx& c) {
  if (!c.h->solver) {
    rocblas_handle r = nullptr;
    if (rocblas_create_handle(&r) != rocblas_status_success) return nullptr;
    c.h->solver = r;
  }
  rocblas_handle r = static_cast<rocblas_handle>(c.h->solver);
  rocblas_set_stream(r, c.s);
  return r;
}

hipError_t gemm_nt64(const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
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
  return gemm_nt(ITN_P_F64, D_F64, g, s);
}

// out[c][r] = in[r*ld + c] for r < rows, c < cols (FP64 strided transpose)
hipError_t transpose_sub(const double* in, int64_t ld, double* out, int64_t rows, int64_t cols, hipStream_t s) {
  const int64_t dims[2] = {cols, rows};
  const int64_t st[2] = {1, ld};
  return permute_cast(D_F64, in, D_F64, out, 2, dims, st, s);
}

// Strided copies collected and run as one launch.  The table goes up with a
// blocking copy: each table buffer is read by one phase of the bond split,
// and a host wait on the stream separates its last readers from the next
// upload (the split's own wait for the eigenvalues, the eigensolver's).
struct CopyList {
  std::vector<Copy2D> items;
  std::vector<PermChunk> chunks;
  void add(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows, int64_t cols) {
    if (rows <= 0 || cols <= 0) return;
    items.push_back(Copy2D{src, dst, rows, cols, lds, ldd});
    for (int64_t f = 0; f < rows * cols; f += PERM_CHUNK)
      chunks.push_back(PermChunk{(int32_t)items.size() - 1, 0, f});
  }
  itn_status run(QCtx& c, DBuf& tab) {
    if (chunks.empty()) return ITN_OK;
    const size_t bi = items.size() * sizeof(Copy2D), bc = chunks.size() * sizeof(PermChunk);
    std::vector<char> host(bi + bc);
    std::memcpy(host.data(), items.data(), bi);
    std::memcpy(host.data() + bi, chunks.data(), bc);
    ITN_TRY(tab.ensure(c.h, bi + bc));
    ITN_HIP(c.h, hipMemcpy(tab.p, host.data(), bi + bc, hipMemcpyHostToDevice));
    const char* d = static_cast<const char*>(tab.p);
    ITN_HIP(c.h, copy2d_batch(reinterpret_cast<const Copy2D*>(d), reinterpret_cast<const PermChunk*>(d + bi),
                              (int64_t)chunks.size(), c.s));
    items.clear();
    chunks.clear();
    return ITN_OK;
  }
};

// Split psi (block-sparse [a, s1, s2, b]) at bond i into sites i, i+1, sector
// by sector of the new link charge q = q(a) + q(s1).
itn_status split(QCtx& c, int i, bool to_right, const QBT& psi, int maxdim, double cutoff, double* trunc) {
  itn_qn_mps* m = c.m;
  const QSpace &sa = psi.q.sp[0], &s1 = psi.q.sp[1], &s2 = psi.q.sp[2], &sb = psi.q.sp[3];
  const auto& mod = m->mod;
  // sectors of the new link: rows (ka, k1) and columns (k2, kb) per charge
  struct Sec {
    std::vector<int32_t> q;
    std::vector<std::pair<int, int>> rows, cols;  // sector pairs, in order
    std::vector<int64_t> roff, coff;
    int64_t nr = 0, nc = 0;
  };
  std::map<std::vector<int32_t>, Sec> secs;
  for (int ka = 0; ka < sa.nsec; ++ka)
    for (int k1 = 0; k1 < s1.nsec; ++k1) {
      auto q = qadd(sa.q(ka), s1.q(k1), mod, +1);
      Sec& S = secs[q];
      S.q = q;
      S.rows.push_back({ka, k1});
      S.roff.push_back(S.nr);
      S.nr += (int64_t)sa.dim[ka] * s1.dim[k1];
    }
  for (int k2 = 0; k2 < s2.nsec; ++k2)
    for (int kb = 0; kb < sb.nsec; ++kb) {
      auto q = qadd(sb.q(kb), s2.q(k2), mod, -1);
      auto it = secs.find(q);
      if (it == secs.end()) continue;
      Sec& S = it->second;
      S.cols.push_back({k2, kb});
      S.coff.push_back(S.nc);
      S.nc += (int64_t)s2.dim[k2] * sb.dim[kb];
    }
  rocblas_handle rb = solver(c);
  if (!rb) return fail(c.h, ITN_E_HIP, "rocblas handle creation failed");
  // per sector: M_q, its density matrix and eigenpairs (ascending); weights to host
  struct Eig {
    Sec* S;
    int64_t n;        // density-matrix dimension
    int64_t mat_off;  // M_q in m->mat
    int64_t rho_off;  // eigenvectors (row j = eigenvector j) in m->rho
    std::vector<double> w;
  };
  std::vector<Eig> eig;
  int64_t mat_tot = 0, rho_tot = 0, ev_tot = 0;
  for (auto& kv : secs) {
    Sec& S = kv.second;
    if (S.nr == 0 || S.nc == 0) continue;
    const int64_t n = to_right ? S.nr : S.nc;
    eig.push_back(Eig{&S, n, mat_tot, rho_tot, {}});
    mat_tot += S.nr * S.nc;
    rho_tot += n * n;
    ev_tot += 2 * n;
  }
  if (eig.empty()) return fail(c.h, ITN_E_ARG, "zero two-site state at bond %d", i);
  ITN_TRY(m->mat.ensure(c.h, mat_tot * 8));
  ITN_TRY(m->matT.ensure(c.h, mat_tot * 8));
  ITN_TRY(m->rho.ensure(c.h, rho_tot * 8));
  ITN_TRY(m->prod.ensure(c.h, mat_tot * 8));
  ITN_TRY(m->ev.ensure(c.h, ev_tot * 8));
  ITN_TRY(m->info.ensure(c.h, 64 + eig.size() * sizeof(rocblas_int)));
  int64_t evo = 0;
  CopyList cpy;
  for (size_t e = 0; e < eig.size(); ++e) {  // gather psi blocks into M_q [nr][nc]
    Sec& S = *eig[e].S;
    double* M = m->mat.d() + eig[e].mat_off;
    for (size_t r = 0; r < S.rows.size(); ++r)
      for (size_t cc = 0; cc < S.cols.size(); ++cc) {
        const std::vector<int32_t> blk = {S.rows[r].first, S.rows[r].second, S.cols[cc].first,
                                          S.cols[cc].second};
        auto it = psi.q.index.find(blk);
        if (it == psi.q.index.end()) return fail(c.h, ITN_E_FLUX, "internal: psi block missing");
        const int64_t br = (int64_t)sa.dim[blk[0]] * s1.dim[blk[1]];
        const int64_t bc = (int64_t)s2.dim[blk[2]] * sb.dim[blk[3]];
        cpy.add(psi.d() + psi.q.off[it->second], bc, M + S.roff[r] * S.nc + S.coff[cc], S.nc, br, bc);
      }
  }
  ITN_TRY(cpy.run(c, m->ctab[0]));
  for (size_t e = 0; e < eig.size(); ++e) {
    Sec& S = *eig[e].S;
    double* M = m->mat.d() + eig[e].mat_off;
    double* rho = m->rho.d() + eig[e].rho_off;
    const int64_t n = eig[e].n;
    if (to_right) {
      ITN_HIP(c.h, gemm_nt64(M, S.nc, M, S.nc, rho, n, n, n, S.nc, c.s));  // M M^T
    } else {
      double* MT = m->matT.d() + eig[e].mat_off;
      ITN_HIP(c.h, transpose_sub(M, S.nc, MT, S.nr, S.nc, c.s));
      ITN_HIP(c.h, gemm_nt64(MT, S.nr, MT, S.nr, rho, n, n, n, S.nr, c.s));  // M^T M
    }
  }
  // The sectors' eigenproblems in a few batched divide-and-conquer calls:
  // sectors sorted by dimension and grouped so that a group's largest is at
  // most 4 times its smallest, each density matrix padded to its group's
  // largest dimension (the padding is a -1 diagonal block, below every
  // weight; its eigenvectors stay in the padding), then each sector's
  // eigenvalues and eigenvectors copied out.  A bond of the Hubbard cylinder
  // has tens of sectors; one solver call each cost more than the solves.
  const int nb = (int)eig.size();
  std::vector<int> order(nb), pos_of(nb);
  std::vector<int64_t> evo_of(nb);
  for (int e = 0; e < nb; ++e) order[e] = e, evo_of[e] = evo, evo += 2 * eig[e].n;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return eig[a].n < eig[b].n; });
  {
    std::vector<int64_t> meta;
    std::vector<std::pair<int, int>> groups;  // [p0, p1) in `order`
    size_t abytes = 0, wbytes = 0;
    for (int p = 0; p < nb;) {
      int q = p + 1;
      while (q < nb && eig[order[q]].n <= eig[order[p]].n * 4) ++q;
      groups.push_back({p, q});
      const int64_t nmax = eig[order[q - 1]].n;
      abytes += (size_t)(q - p) * nmax * nmax * 8;
      wbytes += (size_t)(q - p) * nmax * 2 * 8;
      p = q;
    }
    for (int p = 0; p < nb; ++p) {
      pos_of[order[p]] = p;
      meta.push_back(eig[order[p]].n);
      meta.push_back(eig[order[p]].rho_off);
    }
    ITN_TRY(m->bmeta.ensure(c.h, meta.size() * 8));
    ITN_TRY(m->bat.ensure(c.h, abytes));
    ITN_TRY(m->batw.ensure(c.h, wbytes));
    ITN_HIP(c.h, hipMemcpy(m->bmeta.p, meta.data(), meta.size() * 8, hipMemcpyHostToDevice));
    double* Ab = m->bat.d();
    double* Wb = m->batw.d();
    for (const auto& g : groups) {
      const int cnt = g.second - g.first;
      const int64_t nmax = eig[order[g.second - 1]].n;
      double* Eb = Wb + (size_t)cnt * nmax;
      ITN_HIP(c.h, pad_batch(m->rho.d(), static_cast<const int64_t*>(m->bmeta.p) + 2 * g.first, Ab, nmax,
                             cnt, c.s));
      rocblas_status st = rocsolver_dsyevd_strided_batched(
          rb, rocblas_evect_original, rocblas_fill_upper, (rocblas_int)nmax, Ab, (rocblas_int)nmax,
          (rocblas_stride)(nmax * nmax), Wb, (rocblas_stride)nmax, Eb, (rocblas_stride)nmax,
          static_cast<rocblas_int*>(m->info.p) + g.first, (rocblas_int)cnt);
      if (st != rocblas_status_success)
        return fail(c.h, ITN_E_HIP, "rocsolver_dsyevd_strided_batched failed (%d)", (int)st);
      for (int k = 0; k < cnt; ++k) {
        const int e = order[g.first + k];
        const int64_t n = eig[e].n, lo = nmax - n;  // the sector's eigenpairs are the top n
        cpy.add(Wb + (size_t)k * nmax + lo, 0, m->ev.d() + evo_of[e], 0, 1, n);
        // column lo + j of the padded matrix (rows < n) -> row j of the sector's eigenvectors
        cpy.add(Ab + (size_t)k * nmax * nmax + lo * nmax, nmax, m->rho.d() + eig[e].rho_off, n, n, n);
      }
      Ab += (size_t)cnt * nmax * nmax;
      Wb += (size_t)cnt * nmax * 2;
    }
    // after every group's solve: the copies write over density matrices the padding read
    ITN_TRY(cpy.run(c, m->ctab[1]));
  }
  // eigenvalues and solver status to host
  ITN_TRY(m->pin.ensure(c.h, ev_tot * 8 + eig.size() * sizeof(rocblas_int) + 64));
  char* pin = static_cast<char*>(m->pin.p);
  ITN_HIP(c.h, hipMemcpyAsync(pin, m->ev.p, ev_tot * 8, hipMemcpyDeviceToHost, c.s));
  ITN_HIP(c.h, hipMemcpyAsync(pin + ev_tot * 8, m->info.p, eig.size() * sizeof(rocblas_int),
                              hipMemcpyDeviceToHost, c.s));
  ITN_HIP(c.h, hipStreamSynchronize(c.s));
  evo = 0;
  for (size_t e = 0; e < eig.size(); ++e) {
    rocblas_int inf = 0;  // the solver status of sector e is at its position in the sorted order
    std::memcpy(&inf, pin + ev_tot * 8 + pos_of[e] * sizeof(rocblas_int), sizeof(inf));
    if (inf != 0) return fail(c.h, ITN_E_NOT_CONVERGED, "symmetric eigensolver info=%d at bond %d", (int)inf, i);
    const int64_t n = eig[e].n;
    const double* D = reinterpret_cast<const double*>(pin) + evo;
    // the largest min(rows, cols) eigenvalues are the sector's squared singular values
    const int64_t nsv = std::min(eig[e].S->nr, eig[e].S->nc);
    for (int64_t j = 0; j < nsv; ++j) eig[e].w.push_back(std::max(D[n - 1 - j], 0.0));
    evo += 2 * n;
  }
  // global truncation over all sectors (Sec. 5): weights sorted descending,
  // ties by sector order then position
  struct Wt {
    double w;
    int e, j;
  };
  std::vector<Wt> all;
  double tot = 0.0;
  for (size_t e = 0; e < eig.size(); ++e)
    for (size_t j = 0; j < eig[e].w.size(); ++j) {
      all.push_back(Wt{eig[e].w[j], (int)e, (int)j});
      tot += eig[e].w[j];
    }
  if (!(tot > 0)) return fail(c.h, ITN_E_ARG, "zero two-site state at bond %d", i);
  std::stable_sort(all.begin(), all.end(), [](const Wt& a, const Wt& b) { return a.w > b.w; });
  std::vector<double> pd(all.size());
  for (size_t k = 0; k < all.size(); ++k) pd[k] = all[k].w / tot;
  const int keep = truncation_keep(pd, cutoff, maxdim, c.p->mindim, trunc);
  std::vector<int> kq(eig.size(), 0);
  double kept = 0.0;
  for (int k = 0; k < keep; ++k) {
    kq[all[k].e]++;
    kept += all[k].w;
  }
  const double inv = 1.0 / std::sqrt(kept);
  // the new link: sectors with kept states, in ascending QN order (secs is ordered by QN)
  QSpace nl;
  nl.nq = m->nq;
  nl.mod = mod;
  nl.arrow = +1;
  std::vector<int> e_of_sector;
  for (size_t e = 0; e < eig.size(); ++e)
    if (kq[e] > 0) {
      nl.qn.insert(nl.qn.end(), eig[e].S->q.begin(), eig[e].S->q.end());
      nl.dim.push_back(kq[e]);
      e_of_sector.push_back((int)e);
      nl.nsec++;
    }
  nl.off.resize(nl.nsec);
  nl.total = 0;
  for (int k = 0; k < nl.nsec; ++k) nl.off[k] = nl.total, nl.total += nl.dim[k];
  // new sites: A_i [a:Out, s1:Out, l:In], A_{i+1} [l:Out, s2:Out, b:In]
  std::vector<std::vector<int32_t>> ba, bb;
  for (int k = 0; k < nl.nsec; ++k) {
    const Sec& S = *eig[e_of_sector[k]].S;
    for (auto& r : S.rows) ba.push_back({r.first, r.second, k});
    for (auto& cc : S.cols) bb.push_back({k, cc.first, cc.second});
  }
  std::sort(ba.begin(), ba.end());
  std::sort(bb.begin(), bb.end());
  QBT& Ai = m->A[i];
  QBT& Aj = m->A[i + 1];
  Ai.q = make_qt({with_arrow(sa, +1), with_arrow(s1, +1), with_arrow(nl, -1)}, ba);
  Aj.q = make_qt({with_arrow(nl, +1), with_arrow(s2, +1), with_arrow(sb, -1)}, bb);
  Ai.flux.assign(m->nq, 0);
  Aj.flux.assign(m->nq, 0);
  ITN_TRY(Ai.data.ensure(c.h, std::max<int64_t>(Ai.q.elems, 1) * 8));
  ITN_TRY(Aj.data.ensure(c.h, std::max<int64_t>(Aj.q.elems, 1) * 8));
  int64_t ut_tot = 0;
  for (int k = 0; k < nl.nsec; ++k) ut_tot += (int64_t)kq[e_of_sector[k]] * eig[e_of_sector[k]].n;
  ITN_TRY(m->ut.ensure(c.h, std::max<int64_t>(ut_tot, 1) * 8));
  int64_t uo = 0;
  for (int k = 0; k < nl.nsec; ++k) {  // Ut [kk][n]: kept eigenvectors, largest first (rows reversed)
    const Eig& E = eig[e_of_sector[k]];
    const int64_t n = E.n, kk = kq[e_of_sector[k]];
    cpy.add(m->rho.d() + E.rho_off + (n - 1) * n, -n, m->ut.d() + uo, n, kk, n);
    uo += kk * n;
  }
  ITN_TRY(cpy.run(c, m->ctab[2]));
  uo = 0;
  for (int k = 0; k < nl.nsec; ++k) {
    const Eig& E = eig[e_of_sector[k]];
    const Sec& S = *E.S;
    const int64_t n = E.n, kk = kq[e_of_sector[k]];
    double* Ut = m->ut.d() + uo;
    const double* M = m->mat.d() + E.mat_off;
    double* P = m->prod.d() + E.mat_off;  // kk x nc (right) or nr x kk (left)
    if (to_right) {
      // A_i rows of U (left-orthonormal); A_{i+1} = U^T M / |S_kept|
      double* MT = m->matT.d() + E.mat_off;
      ITN_HIP(c.h, transpose_sub(M, S.nc, MT, S.nr, S.nc, c.s));
      ITN_HIP(c.h, gemm_nt64(Ut, n, MT, S.nr, P, S.nc, kk, S.nc, S.nr, c.s));
      ITN_HIP(c.h, scale(P, inv, kk * S.nc, c.s));
      for (size_t r = 0; r < S.rows.size(); ++r) {
        const std::vector<int32_t> blk = {S.rows[r].first, S.rows[r].second, k};
        const int64_t br = (int64_t)sa.dim[blk[0]] * s1.dim[blk[1]];
        ITN_HIP(c.h, transpose_sub(Ut + S.roff[r], n, Ai.d() + Ai.q.off[Ai.q.index.at(blk)], kk, br, c.s));
      }
      for (size_t cc = 0; cc < S.cols.size(); ++cc) {
        const std::vector<int32_t> blk = {k, S.cols[cc].first, S.cols[cc].second};
        const int64_t bc = (int64_t)s2.dim[blk[1]] * sb.dim[blk[2]];
        cpy.add(P + S.coff[cc], S.nc, Aj.d() + Aj.q.off[Aj.q.index.at(blk)], bc, kk, bc);
      }
    } else {
      // A_{i+1} rows of V^T (right-orthonormal); A_i = M V / |S_kept|
      ITN_HIP(c.h, gemm_nt64(M, S.nc, Ut, n, P, kk, S.nr, kk, S.nc, c.s));
      ITN_HIP(c.h, scale(P, inv, S.nr * kk, c.s));
      for (size_t r = 0; r < S.rows.size(); ++r) {
        const std::vector<int32_t> blk = {S.rows[r].first, S.rows[r].second, k};
        const int64_t br = (int64_t)sa.dim[blk[0]] * s1.dim[blk[1]];
        cpy.add(P + S.roff[r] * kk, kk, Ai.d() + Ai.q.off[Ai.q.index.at(blk)], kk, br, kk);
      }
      for (size_t cc = 0; cc < S.cols.size(); ++cc) {
        const std::vector<int32_t> blk = {k, S.cols[cc].first, S.cols[cc].second};
        const int64_t bc = (int64_t)s2.dim[blk[1]] * sb.dim[blk[2]];
        cpy.add(Ut + S.coff[cc], n, Aj.d() + Aj.q.off[Aj.q.index.at(blk)], bc, kk, bc);
      }
    }
    uo += kk * n;
  }
  ITN_TRY(cpy.run(c, m->ctab[3]));
  m->link[i + 1] = nl;
  return ITN_OK;
}

// An H_eff plan of one bond at one precision, applied with environments
// prepared once.
struct BondPlan {
  itn_plan* pl = nullptr;
  ~BondPlan() {
    if (pl) itn_plan_destroy(pl);
  }
};

// The bond's H_eff plans: FP64 (restarts, refinement) and, below FP64, one at
// `prec` derived from the same structure tables; each applied with its
// environments prepared once (the low-precision ones cast first).
itn_status make_plans(QCtx& c, int i, const QBT& psi, int prec, int nv, BondPlan& p64, BondPlan& plo) {
  itn_qn_mps* m = c.m;
  const QSpace wl = c.mlink, ws = m->site;
  QTensor wq;
  wq.rank = 4;
  wq.sp = {with_arrow(wl, +1), with_arrow(wl, -1), with_arrow(ws, +1), with_arrow(ws, -1)};
  View w1(wq, {}, c.mpo->site(i), ITN_F64), w2(wq, {}, c.mpo->site(i + 1), ITN_F64);
  w1.t.nblocks = w2.t.nblocks = 0;
  w1.t.block_sec = w2.t.block_sec = nullptr;
  w1.t.block_off = w2.t.block_off = nullptr;
  const QBT &L = m->L[i], &R = m->R[i + 2];
  View vl(L.q, L.flux, L.d(), ITN_F64), vr(R.q, R.flux, R.d(), ITN_F64);
  View vp(psi.q, psi.flux, psi.d(), ITN_F64);
  const bool low = prec != ITN_P_F64;
  ITN_TRY(itn_qn_heff_plan(c.h, &vl.t, &w1.t, &w2.t, &vr.t, &vp.t, nv, ITN_P_F64, &p64.pl));
  if (low) ITN_TRY(qn_plan_at_prec(c.h, p64.pl, prec, &plo.pl));
  ITN_TRY(qn_plan_set_direct(p64.pl, 0, 0));
  ITN_TRY(itn_qn_prepare_env(c.h, p64.pl, &vl.t, &vr.t, c.s));
  if (low) {
    const itn_dtype et = prec == ITN_P_BF16 ? ITN_BF16 : ITN_F32;
    const int dt = prec == ITN_P_BF16 ? D_BF16 : D_F32;
    ITN_TRY(m->Lp.ensure(c.h, std::max<int64_t>(L.q.elems, 1) * 4 + 256));
    ITN_TRY(m->Rp.ensure(c.h, std::max<int64_t>(R.q.elems, 1) * 4 + 256));
    ITN_HIP(c.h, cast(D_F64, L.d(), dt, m->Lp.p, L.q.elems, c.s));
    ITN_HIP(c.h, cast(D_F64, R.d(), dt, m->Rp.p, R.q.elems, c.s));
    View ll(L.q, L.flux, m->Lp.p, et), lr(R.q, R.flux, m->Rp.p, et);
    ITN_TRY(qn_plan_set_direct(plo.pl, 0, 0));
    ITN_TRY(itn_qn_prepare_env(c.h, plo.pl, &ll.t, &lr.t, c.s));
  }
  return ITN_OK;
}

// The diagonal of the two-site H_eff at bond i for the block expansion's
// preconditioner, into m->hdiag (psi's block layout); `diag` holds the host
// tables until the solve's first host wait.
itn_status qn_diag(QCtx& c, int i, const QBT& psi, HeffDiag& diag) {
  itn_qn_mps* m = c.m;
  const QBT &L = m->L[i], &R = m->R[i + 2];
  ITN_TRY(heff_diag_build(c.h, L.q, R.q, c.mpo->site(i), c.mpo->site(i + 1), c.mpo->w, psi.q, diag));
  ITN_TRY(m->dtab.ensure(c.h, diag.device_bytes()));
  ITN_TRY(m->hdiag.ensure(c.h, (size_t)std::max<int64_t>(psi.q.elems, 1) * 8));
  ITN_HIP(c.h, heff_diag_launch(diag, L.d(), R.d(), m->dtab.p, m->hdiag.d(), c.s));
  return ITN_OK;
}

itn_status bond_step(QCtx& c, int i, bool to_right, int maxdim, double cutoff, bool last, double* energy,
                     double* trunc) {
  itn_qn_mps* m = c.m;
  QBT& psi = m->theta;  // buffer kept between bonds
  ITN_TRY(contract(c, m->A[i], {1, 2, 3}, false, m->A[i + 1], {3, 4, 5}, false, {1, 2, 4, 5}, psi, true));
  const int64_t n = psi.q.elems;
  const int prec = c.p->prec;
  // block Davidson: plans for B vectors per launch; calls with fewer are padded with zero vectors
  const int B = c.p->block > 1 ? std::min(c.p->block, 8) : 1;
  BondPlan p64, plo;
  ITN_TRY(make_plans(c, i, psi, prec, B, p64, plo));
  if (B > 1) {
    ITN_TRY(m->bx.ensure(c.h, (size_t)B * std::max<int64_t>(n, 1) * 8));
    ITN_TRY(m->by.ensure(c.h, (size_t)B * std::max<int64_t>(n, 1) * 8));
  }
  View vp(psi.q, psi.flux, nullptr, ITN_F64), vo(psi.q, psi.flux, nullptr, ITN_F64);
  const Matvec mv = [&](int p, const double* x, double* y, int nv) -> itn_status {
    for (int v0 = 0; v0 < nv; v0 += B) {
      const int k = std::min(B, nv - v0);
      const double* xs = x + (size_t)v0 * n;
      double* ys = y + (size_t)v0 * n;
      if (k < B) {
        ITN_HIP(c.h, hipMemcpyAsync(m->bx.p, xs, (size_t)k * n * 8, hipMemcpyDeviceToDevice, c.s));
        ITN_HIP(c.h, hipMemsetAsync(m->bx.d() + (size_t)k * n, 0, (size_t)(B - k) * n * 8, c.s));
        xs = m->bx.d();
      }
      vp.t.data = const_cast<double*>(xs);
      vo.t.data = k < B ? m->by.d() : ys;
      ITN_TRY(itn_qn_heff_apply(c.h, p == ITN_P_F64 ? p64.pl : plo.pl, nullptr, nullptr, &vp.t, &vo.t, c.s));
      if (k < B)
        ITN_HIP(c.h, hipMemcpyAsync(ys, m->by.p, (size_t)k * n * 8, hipMemcpyDeviceToDevice, c.s));
    }
    return ITN_OK;
  };
  HeffDiag diag_tables;  // read by the diagonal's upload; alive until the solve's host waits
  const double* diag = nullptr;
  if (B > 1) {
    ITN_TRY(qn_diag(c, i, psi, diag_tables));
    diag = m->hdiag.d();
  }
  const double tol = c.p->eig_tol > 0 ? c.p->eig_tol : 1e-10;
  const int maxiter = c.p->maxiter > 0 ? c.p->maxiter : 100;
  double e = 0.0, r = 0.0;
  bool conv = true;
  {
    PhaseTimer pt(c, &c.t_solve);
    // A tiny reproducible component in every allowed block of the start
    // vector: a symmetric product start (Neel) can otherwise leave the Krylov
    // space inside a symmetry subspace of H_eff that misses the ground state.
    ITN_HIP(c.h, add_noise(psi.d(), n, 1e-7 / std::sqrt((double)std::max<int64_t>(n, 1)),
                           0x5eedull * 1000003ull + (uint64_t)(c.sweep * 4096 + i * 2 + (to_right ? 0 : 1)),
                           c.s));
    ITN_TRY(davidson(c, mv, prec, tol, maxiter, psi.d(), n, diag, last, &e, &r, &conv));
  }
  c.max_resid = std::max(c.max_resid, r);
  if (!conv && (prec == ITN_P_F64 || c.p->refine)) c.unconverged = true;
  *energy = e;
  {
    PhaseTimer pt(c, &c.t_split);
    ITN_TRY(split(c, i, to_right, psi, maxdim, cutoff, trunc));
  }
  PhaseTimer pt(c, &c.t_env);
  if (to_right) return env_step(c, i, true);
  return env_step(c, i + 1, false);
}

}  // namespace

extern "C" {

itn_status itn_qn_mps_create(itn_handle* h, int32_t N, int32_t d, int32_t nq, const int32_t* site_qn,
                             const int32_t* mod, const int32_t* state, itn_qn_mps** out) {
  if (!h || !out || !site_qn || !state) return h ? fail(h, ITN_E_ARG, "null argument") : ITN_E_ARG;
  *out = nullptr;
  if (N < 2 || d < 1 || nq < 1) return fail(h, ITN_E_ARG, "need N >= 2, d >= 1, nq >= 1");
  if (h->device < 0) return fail(h, ITN_E_NODEVICE, "host-only handle cannot hold an MPS");
  std::vector<int32_t> md(nq, 0);
  if (mod)
    for (int c = 0; c < nq; ++c) {
      if (mod[c] < 0 || mod[c] == 1) return fail(h, ITN_E_ARG, "a QN addition rule is 0 or N >= 2");
      md[c] = mod[c];
    }
  for (int i = 0; i < N; ++i)
    if (state[i] < 0 || state[i] >= d) return fail(h, ITN_E_ARG, "state[%d] out of range", i);
  auto* m = new itn_qn_mps();
  m->N = N;
  m->d = d;
  m->nq = nq;
  m->mod = md;
  m->site = space_from_basis(site_qn, d, nq, md, +1);
  m->link.resize(N + 1);
  m->A.resize(N);
  m->L.resize(N + 1);
  m->R.resize(N + 1);
  std::vector<int32_t> q(nq, 0);
  m->link[0] = single_sector(q, md, +1);
  for (int i = 0; i < N; ++i) {
    auto nq_ = qadd(q.data(), site_qn + (size_t)state[i] * nq, md, +1);
    m->link[i + 1] = single_sector(nq_, md, +1);
    const auto loc = locate(m->site, state[i]);
    QBT& A = m->A[i];
    A.q = make_qt({with_arrow(m->link[i], +1), m->site, with_arrow(m->link[i + 1], -1)}, {{0, loc.first, 0}});
    A.flux.assign(nq, 0);
    std::vector<double> v(m->site.dim[loc.first], 0.0);
    v[loc.second] = 1.0;
    itn_status st = upload(h, A, v);
    if (st != ITN_OK) {
      delete m;
      return st;
    }
    q = nq_;
  }
  *out = m;
  return ITN_OK;
}

itn_status itn_qn_mps_destroy(itn_qn_mps* m) {
  if (m) (void)hipDeviceSynchronize();
  delete m;
  return ITN_OK;
}

itn_status itn_qn_mps_bonds(const itn_qn_mps* m, int32_t* bond) {
  if (!m || !bond) return ITN_E_ARG;
  for (int i = 0; i <= m->N; ++i) bond[i] = (int32_t)m->link[i].total;
  return ITN_OK;
}

itn_status itn_qn_mps_get_site(itn_handle* h, const itn_qn_mps* m, int32_t i, double* host) {
  if (!h || !m || !host) return ITN_E_ARG;
  if (i < 0 || i >= m->N) return fail(h, ITN_E_ARG, "site index out of range");
  const QBT& A = m->A[i];
  std::vector<double> blocks(std::max<int64_t>(A.q.elems, 1));
  ITN_HIP(h, hipDeviceSynchronize());
  if (A.q.elems > 0) ITN_HIP(h, hipMemcpy(blocks.data(), A.d(), A.q.elems * 8, hipMemcpyDeviceToHost));
  const int64_t n0 = A.q.sp[0].total, n1 = A.q.sp[1].total, n2 = A.q.sp[2].total;
  std::fill(host, host + n0 * n1 * n2, 0.0);
  for (size_t b = 0; b < A.q.blocks.size(); ++b) {
    const auto& k = A.q.blocks[b];
    const int64_t d0 = A.q.sp[0].dim[k[0]], d1 = A.q.sp[1].dim[k[1]], d2 = A.q.sp[2].dim[k[2]];
    const int64_t o0 = A.q.sp[0].off[k[0]], o1 = A.q.sp[1].off[k[1]], o2 = A.q.sp[2].off[k[2]];
    const double* src = blocks.data() + A.q.off[b];
    for (int64_t x = 0; x < d0; ++x)
      for (int64_t y = 0; y < d1; ++y)
        for (int64_t z = 0; z < d2; ++z)
          host[((o0 + x) * n1 + (o1 + y)) * n2 + (o2 + z)] = src[(x * d1 + y) * d2 + z];
  }
  return ITN_OK;
}

itn_status itn_qn_mps_link(const itn_qn_mps* m, int32_t k, int32_t* nsec, int32_t* qn, int32_t* dim) {
  if (!m || !nsec || k < 0 || k > m->N) return ITN_E_ARG;
  const QSpace& s = m->link[k];
  if (qn && dim && *nsec >= s.nsec) {
    std::copy(s.qn.begin(), s.qn.end(), qn);
    std::copy(s.dim.begin(), s.dim.end(), dim);
  }
  *nsec = s.nsec;
  return ITN_OK;
}

itn_status itn_qn_dmrg_sweep(itn_handle* h, itn_qn_mps* mps, const itn_mpo* mpo, const int32_t* link_qn,
                             const itn_sweep_params* p, itn_sweep_result* res) {
  if (!h || !mps || !mpo || !p || !link_qn) return h ? fail(h, ITN_E_ARG, "null argument") : ITN_E_ARG;
  if (mpo->N != mps->N || mpo->d != mps->d)
    return fail(h, ITN_E_SHAPE, "MPO (N=%d, d=%d) does not match the MPS (N=%d, d=%d)", mpo->N, mpo->d,
                mps->N, mps->d);
  if (p->nsweeps < 0 || (p->nsweeps > 0 && (!p->maxdim || !p->cutoff)))
    return fail(h, ITN_E_ARG, "bad sweep schedule");
  if (p->prec != ITN_P_F64 && p->prec != ITN_P_F32 && p->prec != ITN_P_BF16)
    return fail(h, ITN_E_ARG, "unknown precision");
  if (p->northo > 0) return fail(h, ITN_E_UNSUPPORTED, "excited states are not supported on QN sweeps");
  for (int k = 0; k < p->nsweeps; ++k)
    if (p->maxdim[k] < 1 || p->cutoff[k] < 0) return fail(h, ITN_E_ARG, "bad maxdim/cutoff");
  if (h->device < 0) return fail(h, ITN_E_NODEVICE, "host-only handle cannot run sweeps");
  QCtx c;
  c.h = h;
  c.p = p;
  c.sb = &mps->sb;
  c.m = mps;
  c.mpo = mpo;
  const int N = mps->N, w = mpo->w, d = mpo->d, nq = mps->nq;
  c.mlink = space_from_basis(link_qn, w, nq, mps->mod, +1);
  // MPO sites as block tensors; entries outside the flux-allowed blocks are an error
  c.W.resize(N);
  QTensor wq;
  wq.rank = 4;
  wq.sp = {with_arrow(c.mlink, +1), with_arrow(c.mlink, -1), with_arrow(mps->site, +1),
           with_arrow(mps->site, -1)};
  const auto wblocks = allowed_blocks(wq);
  for (int i = 0; i < N; ++i) {
    const double* Wd = mpo->site(i);
    QBT& W = c.W[i];
    W.q = make_qt(wq.sp, wblocks);
    W.flux.assign(nq, 0);
    std::vector<double> host(std::max<int64_t>(W.q.elems, 1), 0.0);
    std::vector<char> covered((size_t)w * w * d * d, 0);
    for (size_t b = 0; b < W.q.blocks.size(); ++b) {
      const auto& k = W.q.blocks[b];
      const int64_t D0 = W.q.sp[0].dim[k[0]], D1 = W.q.sp[1].dim[k[1]], D2 = W.q.sp[2].dim[k[2]],
                    D3 = W.q.sp[3].dim[k[3]];
      int64_t t = W.q.off[b];
      for (int64_t a = 0; a < D0; ++a)
        for (int64_t bb = 0; bb < D1; ++bb)
          for (int64_t sp_ = 0; sp_ < D2; ++sp_)
            for (int64_t s_ = 0; s_ < D3; ++s_) {
              const int64_t ia = W.q.sp[0].off[k[0]] + a, ib = W.q.sp[1].off[k[1]] + bb,
                            ic = W.q.sp[2].off[k[2]] + sp_, id = W.q.sp[3].off[k[3]] + s_;
              const size_t flat = ((ia * w + ib) * d + ic) * d + id;
              host[t++] = Wd[flat];
              covered[flat] = 1;
            }
    }
    for (size_t f = 0; f < covered.size(); ++f)
      if (!covered[f] && Wd[f] != 0.0)
        return fail(h, ITN_E_FLUX, "MPO site %d has a nonzero entry outside the allowed blocks", i);
    ITN_TRY(upload(h, W, host));
  }
  std::vector<int32_t> lq(link_qn, link_qn + (size_t)w * nq);
  if (!mps->envs || mps->env_mpo != mpo || mps->env_link_qn != lq) {
    // boundaries: L_0 selects channel w-1, R_N channel 0
    std::vector<int32_t> zero(nq, 0);
    const auto lw = locate(c.mlink, w - 1), r0 = locate(c.mlink, 0);
    QBT& L0 = mps->L[0];
    L0.q = make_qt({with_arrow(mps->link[0], +1), with_arrow(c.mlink, -1), with_arrow(mps->link[0], -1)},
                   {{0, lw.first, 0}});
    L0.flux = zero;
    std::vector<double> lv(c.mlink.dim[lw.first], 0.0);
    lv[lw.second] = 1.0;
    ITN_TRY(upload(h, L0, lv));
    QBT& RN = mps->R[N];
    RN.q = make_qt({with_arrow(mps->link[N], -1), with_arrow(c.mlink, +1), with_arrow(mps->link[N], +1)},
                   {{0, r0.first, 0}});
    RN.flux = zero;
    std::vector<double> rv(c.mlink.dim[r0.first], 0.0);
    rv[r0.second] = 1.0;
    ITN_TRY(upload(h, RN, rv));
    if (block_flux(L0.q, L0.q.blocks[0]) != zero || block_flux(RN.q, RN.q.blocks[0]) != zero)
      return fail(h, ITN_E_FLUX, "boundary channels must carry zero charge");
    for (int i = N - 1; i >= 2; --i) ITN_TRY(env_step(c, i, false));
    mps->envs = true;
    mps->env_mpo = mpo;
    mps->env_link_qn = lq;
  }
  if (res) res->sweeps_done = 0;
  double prevE = 0.0;
  for (int sw = 0; sw < p->nsweeps; ++sw) {
    auto t0 = std::chrono::steady_clock::now();
    c.sweep = sw;
    c.matvecs = c.matvecs64 = 0;
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
      int32_t mb = 0;
      for (auto& l : mps->link) mb = std::max<int32_t>(mb, (int32_t)l.total);
      if (res->max_bond) res->max_bond[sw] = mb;
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
