// C ABI of libitn: handle management, labelled contraction, dense H_eff,
// environment update.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <set>

#include "handle.h"

using namespace itn;

namespace itn {

void WTable::release() {
  if (row_ptr) (void)hipFree(row_ptr);
  if (row_off) (void)hipFree(row_off);
  if (col_off) (void)hipFree(col_off);
  if (coef) (void)hipFree(coef);
  if (col_idx) (void)hipFree(col_idx);
  if (coef32) (void)hipFree(coef32);
  col_idx = nullptr;
  coef32 = nullptr;
  row_ptr = nullptr;
  row_off = col_off = nullptr;
  coef = nullptr;
}

itn_status fail(itn_handle* h, itn_status st, const char* fmt, ...) {
  if (h) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    h->err = buf;
  }
  return st;
}

itn_status hip_fail(itn_handle* h, hipError_t e, const char* where) {
  return fail(h, ITN_E_HIP, "HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), where);
}

itn_status ensure_workspace(itn_handle* h, size_t bytes) {
  if (h->ws.query) {
    h->ws.query_bytes = bytes;
    return ITN_STOP_QUERY;
  }
  if (h->device < 0) return fail(h, ITN_E_NODEVICE, "host-only handle cannot launch work");
  if (bytes <= h->ws.size) return ITN_OK;
  if (h->ws.caller)
    return fail(h, ITN_E_WORKSPACE, "this call needs %zu bytes of workspace; the caller's holds %zu",
                bytes, h->ws.size);
  ITN_HIP(h, hipDeviceSynchronize());
  if (h->ws.ptr) ITN_HIP(h, hipFree(h->ws.ptr));
  h->ws.ptr = nullptr;
  h->ws.size = 0;
  size_t want = std::max(bytes, (size_t)1 << 20);
  hipError_t e = hipMalloc(&h->ws.ptr, want);
  if (e != hipSuccess) {
    h->ws.ptr = nullptr;
    return fail(h, ITN_E_WORKSPACE, "workspace allocation of %zu bytes failed", want);
  }
  h->ws.size = want;
  return ITN_OK;
}

static hipEvent_t pool_event(itn_handle* h) {
  if (!h->ev_pool.empty()) {
    hipEvent_t e = h->ev_pool.back();
    h->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

Prof::Prof(itn_handle* h_, const char* n, hipStream_t s_) : h(h_), name(n), s(s_) {
  if (!h->prof_on) return;
  a = pool_event(h);
  b = pool_event(h);
  if (a) (void)hipEventRecord(a, s);
}

Prof::~Prof() {
  if (!h->prof_on || !a || !b) return;
  (void)hipEventRecord(b, s);
  h->prof.push_back(ProfRec{name, a, b});
}

std::string CSR::key() const {
  std::string k;
  auto app = [&](const void* p, size_t n) { k.append(static_cast<const char*>(p), n); };
  size_t sz[4] = {row_ptr.size(), row_off.size(), col_off.size(), coef.size()};
  app(sz, sizeof(sz));
  app(row_ptr.data(), row_ptr.size() * 4);
  app(row_off.data(), row_off.size() * 8);
  app(col_off.data(), col_off.size() * 8);
  app(coef.data(), coef.size() * 8);
  return k;
}

itn_status get_wtable(itn_handle* h, const std::string& key, const std::vector<int32_t>& row_ptr,
                      const std::vector<int64_t>& row_off, const std::vector<int64_t>& col_off,
                      const std::vector<double>& coef, const WTable** out) {
  auto it = h->wtables.find(key);
  if (it != h->wtables.end()) {
    *out = it->second.get();
    return ITN_OK;
  }
  if (h->wtables.size() > 256) {
    ITN_HIP(h, hipDeviceSynchronize());
    for (auto& kv : h->wtables) kv.second->release();
    h->wtables.clear();
  }
  auto t = std::make_unique<WTable>();
  t->nrows = (int32_t)row_off.size();
  t->nnz = (int64_t)coef.size();
  const size_t nz = std::max<size_t>(1, coef.size());
  ITN_HIP(h, hipMalloc(&t->row_ptr, row_ptr.size() * 4));
  ITN_HIP(h, hipMalloc(&t->row_off, std::max<size_t>(1, row_off.size()) * 8));
  ITN_HIP(h, hipMalloc(&t->col_off, nz * 8));
  ITN_HIP(h, hipMalloc(&t->coef, nz * 8));
  ITN_HIP(h, hipMemcpy(t->row_ptr, row_ptr.data(), row_ptr.size() * 4, hipMemcpyHostToDevice));
  if (!row_off.empty())
    ITN_HIP(h, hipMemcpy(t->row_off, row_off.data(), row_off.size() * 8, hipMemcpyHostToDevice));
  ITN_HIP(h, hipMalloc(&t->col_idx, nz * 4));
  ITN_HIP(h, hipMalloc(&t->coef32, nz * 4));
  if (!coef.empty()) {
    ITN_HIP(h, hipMemcpy(t->col_off, col_off.data(), col_off.size() * 8, hipMemcpyHostToDevice));
    ITN_HIP(h, hipMemcpy(t->coef, coef.data(), coef.size() * 8, hipMemcpyHostToDevice));
    std::vector<int32_t> ci(col_off.begin(), col_off.end());
    std::vector<float> cf(coef.begin(), coef.end());
    ITN_HIP(h, hipMemcpy(t->col_idx, ci.data(), ci.size() * 4, hipMemcpyHostToDevice));
    ITN_HIP(h, hipMemcpy(t->coef32, cf.data(), cf.size() * 4, hipMemcpyHostToDevice));
  }
  *out = t.get();
  h->wtables.emplace(key, std::move(t));
  return ITN_OK;
}

}  // namespace itn

// --------------------------------------------------------------- validation
namespace {

bool valid_dtype(int dt) { return dt == ITN_F64 || dt == ITN_F32 || dt == ITN_BF16; }
bool valid_prec(int p) { return p == ITN_P_F64 || p == ITN_P_F32 || p == ITN_P_BF16; }

itn_status check_dense(itn_handle* h, const itn_tensor* t, const char* name, int rank) {
  if (!t) return fail(h, ITN_E_ARG, "%s is NULL", name);
  if (rank >= 0 && t->rank != rank)
    return fail(h, ITN_E_SHAPE, "%s must have rank %d (got %d)", name, rank, t->rank);
  if (t->rank < 0 || t->rank > 8) return fail(h, ITN_E_SHAPE, "%s rank %d out of range", name, t->rank);
  if (t->rank > 0 && !t->dims) return fail(h, ITN_E_ARG, "%s dims is NULL", name);
  if (t->nblocks != 0) return fail(h, ITN_E_ARG, "%s must be dense (nblocks == 0)", name);
  if (!valid_dtype(t->dtype)) return fail(h, ITN_E_DTYPE, "%s has an unknown dtype", name);
  for (int k = 0; k < t->rank; ++k)
    if (t->dims[k] < 0) return fail(h, ITN_E_SHAPE, "%s has a negative extent", name);
  return ITN_OK;
}

int64_t numel(const itn_tensor* t) {
  int64_t n = 1;
  for (int k = 0; k < t->rank; ++k) n *= t->dims[k];
  return n;
}

int xtype_of(int prec) { return prec == ITN_P_F64 ? D_F64 : D_F32; }

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

// CSR of the H_eff W-stage: output (c' = s1' d + s2', m2) <- input
// (m0, c = s1 d + s2), coefficient sum_m1 W1[m0,m1,s1',s1] W2[m1,m2,s2',s2].
CSR heff_w_csr(const double* W1, const double* W2, int w, int d, int64_t in_m_stride,
               int64_t in_c_stride, int64_t out_c_stride, int64_t out_m_stride) {
  CSR csr;
  const int d2 = d * d;
  auto w1 = [&](int a, int b, int sp, int s) { return W1[((a * w + b) * d + sp) * d + s]; };
  auto w2 = [&](int a, int b, int sp, int s) { return W2[((a * w + b) * d + sp) * d + s]; };
  for (int cp = 0; cp < d2; ++cp) {
    const int s1p = cp / d, s2p = cp % d;
    for (int m2 = 0; m2 < w; ++m2) {
      for (int m0 = 0; m0 < w; ++m0)
        for (int c = 0; c < d2; ++c) {
          const int s1 = c / d, s2 = c % d;
          double v = 0.0;
          for (int m1 = 0; m1 < w; ++m1) v += w1(m0, m1, s1p, s1) * w2(m1, m2, s2p, s2);
          if (v != 0.0) {
            csr.col_off.push_back(m0 * in_m_stride + c * in_c_stride);
            csr.coef.push_back(v);
          }
        }
      csr.row_off.push_back(cp * out_c_stride + m2 * out_m_stride);
      csr.row_ptr.push_back((int32_t)csr.coef.size());
    }
  }
  return csr;
}

// CSR of one MPO tensor applied in an environment step: output (mo, sp) <-
// input (mi, s) with coefficient W[m_in, m_out, s', s]; `left` selects
// whether the input channel is the first (left step) or second MPO index.
CSR env_w_csr(const double* W, int w, int d, bool left, int64_t in_m, int64_t in_s, int64_t out_m,
              int64_t out_s) {
  CSR csr;
  for (int mo = 0; mo < w; ++mo)
    for (int sp = 0; sp < d; ++sp) {
      for (int mi = 0; mi < w; ++mi)
        for (int s = 0; s < d; ++s) {
          // left:  T2[.., s', m', ..] = sum_{m, s} T1[m, s] W[m, m', s', s]
          // right: T2[.., m, s', ..]  = sum_{m', s} T1[m', s] W[m, m', s', s]
          const double v = left ? W[((mi * w + mo) * d + sp) * d + s]
                                : W[((mo * w + mi) * d + sp) * d + s];
          if (v != 0.0) {
            csr.col_off.push_back(mi * in_m + s * in_s);
            csr.coef.push_back(v);
          }
        }
      csr.row_off.push_back(mo * out_m + sp * out_s);
      csr.row_ptr.push_back((int32_t)csr.coef.size());
    }
  return csr;
}

}  // namespace

// ------------------------------------------------------------------- handle
extern "C" {

const char* itn_version(void) { return "libitn 0.1 (gfx950)"; }

itn_status itn_create(itn_handle** out, int device) {
  if (!out) return ITN_E_ARG;
  *out = nullptr;
  auto* h = new itn_handle();
  h->device = device;
  if (device >= 0) {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || device >= n) {
      delete h;
      return ITN_E_NODEVICE;
    }
    e = hipSetDevice(device);
    if (e != hipSuccess) {
      delete h;
      return ITN_E_HIP;
    }
    noalloc_scratch_init(device);
  }
  *out = h;
  return ITN_OK;
}

void itn_release_solver(itn_handle* h);  // in api_dmrg.cpp

itn_status itn_destroy(itn_handle* h) {
  if (!h) return ITN_E_ARG;
  if (h->device >= 0) {
    (void)hipDeviceSynchronize();
    for (auto& r : h->prof) (void)hipEventDestroy(r.a), (void)hipEventDestroy(r.b);
    for (auto e : h->ev_pool) (void)hipEventDestroy(e);
    for (auto& kv : h->wtables) kv.second->release();
    if (h->ws.ptr && !h->ws.caller) (void)hipFree(h->ws.ptr);
    itn_release_solver(h);
  }
  delete h;
  return ITN_OK;
}

const char* itn_last_error(const itn_handle* h) { return h ? h->err.c_str() : "null handle"; }

itn_status itn_profile_enable(itn_handle* h, int32_t on) {
  if (!h) return ITN_E_ARG;
  if (h->device < 0) return fail(h, ITN_E_NODEVICE, "host-only handle has no launches to time");
  h->prof_on = on != 0;
  return ITN_OK;
}

itn_status itn_profile_report(itn_handle* h, int32_t max_entries, char* names, double* total_ms,
                              int64_t* count, int32_t* n_entries) {
  if (!h || !n_entries || (max_entries > 0 && (!names || !total_ms || !count))) return ITN_E_ARG;
  if (h->device < 0) return fail(h, ITN_E_NODEVICE, "host-only handle has no launches to time");
  ITN_HIP(h, hipDeviceSynchronize());
  std::vector<std::string> order;
  std::map<std::string, std::pair<double, int64_t>> agg;
  for (auto& r : h->prof) {
    float ms = 0.f;
    ITN_HIP(h, hipEventElapsedTime(&ms, r.a, r.b));
    auto it = agg.find(r.name);
    if (it == agg.end()) {
      order.push_back(r.name);
      agg[r.name] = {ms, 1};
    } else {
      it->second.first += ms;
      it->second.second += 1;
    }
    h->ev_pool.push_back(r.a);
    h->ev_pool.push_back(r.b);
  }
  h->prof.clear();
  const int n = (int)order.size();
  *n_entries = n;
  for (int i = 0; i < n && i < max_entries; ++i) {
    std::snprintf(names + 32 * i, 32, "%s", order[i].c_str());
    total_ms[i] = agg[order[i]].first;
    count[i] = agg[order[i]].second;
  }
  return ITN_OK;
}

itn_status itn_sync(itn_handle* h, void* hip_stream) {
  if (!h) return ITN_E_ARG;
  if (h->device < 0) return ITN_OK;
  ITN_HIP(h, hipStreamSynchronize(as_stream(hip_stream)));
  return ITN_OK;
}

itn_status itn_cast(itn_handle* h, const itn_tensor* src, itn_tensor* dst, void* hip_stream) {
  if (!h) return ITN_E_ARG;
  ITN_TRY(check_dense(h, src, "src", -1));
  ITN_TRY(check_dense(h, dst, "dst", -1));
  if (src->rank != dst->rank) return fail(h, ITN_E_SHAPE, "src and dst ranks differ");
  for (int k = 0; k < src->rank; ++k)
    if (src->dims[k] != dst->dims[k]) return fail(h, ITN_E_SHAPE, "src and dst extents differ");
  if (h->device < 0) return fail(h, ITN_E_NODEVICE, "host-only handle cannot launch work");
  const int64_t n = numel(src);
  if (n == 0) return ITN_OK;
  hipStream_t s = as_stream(hip_stream);
  Prof pf(h, "cast", s);
  ITN_HIP(h, cast(src->dtype, src->data, dst->dtype, dst->data, n, s));
  return ITN_OK;
}

// --------------------------------------------------------------- contract
itn_status itn_contract(itn_handle* h, const itn_tensor* A, const itn_tensor* B, itn_tensor* C,
                        itn_prec prec, void* hip_stream) {
  if (!h) return ITN_E_ARG;
  if (!A || !B || !C) return fail(h, ITN_E_ARG, "A, B and C are required");
  if (A->space || B->space || C->space) return contract_qn(h, A, B, C, prec, hip_stream);
  ITN_TRY(check_dense(h, A, "A", -1));
  ITN_TRY(check_dense(h, B, "B", -1));
  ITN_TRY(check_dense(h, C, "C", -1));
  if (!valid_prec(prec)) return fail(h, ITN_E_ARG, "unknown precision");
  if ((A->rank && !A->label) || (B->rank && !B->label) || (C->rank && !C->label))
    return fail(h, ITN_E_ARG, "labels missing");
  if (C->dtype == ITN_BF16) return fail(h, ITN_E_DTYPE, "C must be F64 or F32");
  auto uniq = [](const itn_tensor* t) {
    std::set<int32_t> s(t->label, t->label + t->rank);
    return (int)s.size() == t->rank;
  };
  if (!uniq(A) || !uniq(B) || !uniq(C)) return fail(h, ITN_E_LABEL, "repeated label in an operand");
  auto find = [](const itn_tensor* t, int32_t l) {
    for (int k = 0; k < t->rank; ++k)
      if (t->label[k] == l) return k;
    return -1;
  };
  std::vector<int> freeA, freeB, conA, conB;
  for (int k = 0; k < A->rank; ++k) {
    const int j = find(B, A->label[k]);
    if (j < 0) freeA.push_back(k);
    else {
      if (A->dims[k] != B->dims[j])
        return fail(h, ITN_E_SHAPE, "contracted label %d has extents %lld and %lld", A->label[k],
                    (long long)A->dims[k], (long long)B->dims[j]);
      conA.push_back(k);
      conB.push_back(j);
    }
  }
  for (int k = 0; k < B->rank; ++k)
    if (find(A, B->label[k]) < 0) freeB.push_back(k);
  if ((int)(freeA.size() + freeB.size()) != C->rank)
    return fail(h, ITN_E_LABEL, "C must carry exactly the uncontracted labels");
  // C index k -> (operand, axis)
  std::vector<int64_t> cdims(C->rank);
  for (int k = 0; k < C->rank; ++k) {
    const int ja = find(A, C->label[k]), jb = find(B, C->label[k]);
    const bool inA = ja >= 0 && find(B, C->label[k]) < 0;
    const bool inB = jb >= 0 && find(A, C->label[k]) < 0;
    if (!inA && !inB) return fail(h, ITN_E_LABEL, "C label %d is not an uncontracted label", C->label[k]);
    cdims[k] = inA ? A->dims[ja] : B->dims[jb];
    if (cdims[k] != C->dims[k])
      return fail(h, ITN_E_SHAPE, "C extent of label %d is %lld, expected %lld", C->label[k],
                  (long long)C->dims[k], (long long)cdims[k]);
  }
  int64_t M = 1, N = 1, K = 1;
  for (int k : freeA) M *= A->dims[k];
  for (int k : freeB) N *= B->dims[k];
  for (int k : conA) K *= A->dims[k];
  if (h->device < 0 && !h->ws.query) return fail(h, ITN_E_NODEVICE, "host-only handle cannot launch work");
  hipStream_t s = as_stream(hip_stream);
  const int64_t nC = numel(C);
  if (nC == 0) return ITN_OK;
  if (M * N != nC) return fail(h, ITN_E_SHAPE, "internal size mismatch");
  const int P = prec;
  const int pt = P == ITN_P_F64 ? D_F64 : (P == ITN_P_F32 ? D_F32 : D_BF16);
  const int es = dtype_size(pt);
  // Is C's label order the natural [freeA..., freeB...] order?
  bool natural = true;
  {
    int k = 0;
    for (int a : freeA) natural &= C->label[k++] == A->label[a];
    for (int b : freeB) natural &= C->label[k++] == B->label[b];
  }
  const int tmp_dt = natural ? C->dtype : (P == ITN_P_F64 ? D_F64 : D_F32);
  const size_t bytesA = round256((size_t)(M * K) * es), bytesB = round256((size_t)(N * K) * es);
  const size_t bytesT = natural ? 0 : round256((size_t)nC * dtype_size(tmp_dt));
  ITN_TRY(ensure_workspace(h, bytesA + bytesB + bytesT + 256));
  Carver cv(h->ws.ptr);
  void* Ap = cv.take(bytesA);
  void* Bp = cv.take(bytesB);
  void* Tp = natural ? C->data : cv.take(bytesT);
  auto strides = [](const itn_tensor* t) {
    std::vector<int64_t> st(t->rank);
    int64_t acc = 1;
    for (int k = t->rank - 1; k >= 0; --k) {
      st[k] = acc;
      acc *= t->dims[k];
    }
    return st;
  };
  const auto sa = strides(A), sb = strides(B);
  if (K == 0) {
    ITN_HIP(h, fill(C->data, C->dtype, 0.0, nC, s));
    return ITN_OK;
  }
  {  // A -> [freeA..., con...]
    std::vector<int64_t> od, is;
    for (int k : freeA) od.push_back(A->dims[k]), is.push_back(sa[k]);
    for (int k : conA) od.push_back(A->dims[k]), is.push_back(sa[k]);
    if (od.empty()) od.push_back(1), is.push_back(0);
    ITN_HIP(h, permute_cast(A->dtype, A->data, pt, Ap, (int)od.size(), od.data(), is.data(), s));
  }
  {  // B -> [freeB..., con (A's order)...]
    std::vector<int64_t> od, is;
    for (int k : freeB) od.push_back(B->dims[k]), is.push_back(sb[k]);
    for (int k : conB) od.push_back(B->dims[k]), is.push_back(sb[k]);
    if (od.empty()) od.push_back(1), is.push_back(0);
    ITN_HIP(h, permute_cast(B->dtype, B->data, pt, Bp, (int)od.size(), od.data(), is.data(), s));
  }
  GemmArgs g{};
  g.A = Ap;
  g.B = Bp;
  g.C = Tp;
  g.M = M;
  g.N = N;
  g.K = K;
  g.lda = K;
  g.ldb = K;
  g.ldc = N;
  g.batch = 1;
  ITN_HIP(h, gemm_nt(P, tmp_dt, g, s));
  if (!natural) {
    // T is [freeA..., freeB...]; gather into C's order.
    std::vector<int64_t> tdims;
    for (int k : freeA) tdims.push_back(A->dims[k]);
    for (int k : freeB) tdims.push_back(B->dims[k]);
    std::vector<int64_t> tstr(tdims.size());
    int64_t acc = 1;
    for (int k = (int)tdims.size() - 1; k >= 0; --k) tstr[k] = acc, acc *= tdims[k];
    std::vector<int64_t> od(C->rank), is(C->rank);
    for (int k = 0; k < C->rank; ++k) {
      int pos = -1;
      for (size_t a = 0; a < freeA.size(); ++a)
        if (A->label[freeA[a]] == C->label[k]) pos = (int)a;
      for (size_t b = 0; b < freeB.size(); ++b)
        if (B->label[freeB[b]] == C->label[k]) pos = (int)(freeA.size() + b);
      od[k] = C->dims[k];
      is[k] = tstr[pos];
    }
    ITN_HIP(h, permute_cast(tmp_dt, Tp, C->dtype, C->data, C->rank, od.data(), is.data(), s));
  }
  return ITN_OK;
}

}  // extern "C"

// -------------------------------------------------------------- dense H_eff
static size_t heff_ws_bytes(int64_t cl, int64_t cr, int d, int w, int nv, int P, bool castL,
                            bool castR) {
  const int es = P == ITN_P_F64 ? 8 : (P == ITN_P_F32 ? 4 : 2);
  const int xs = P == ITN_P_F64 ? 8 : 4;
  const int64_t d2 = (int64_t)d * d;
  size_t b = 0;
  if (castL) b += round256((size_t)(cl * w * cl) * es);
  if (castR) b += round256((size_t)(cr * w * cr) * es);
  b += round256((size_t)(d2 * nv * cr * cl) * es);        // psiT
  b += round256((size_t)(cl * w * d2 * nv * cr) * xs);     // X (unfused path)
  b += round256((size_t)(nv * cl * d2 * w * cr) * es);     // Z
  return b + 256;
}

extern "C" itn_status itn_heff_workspace_size(itn_handle* h, int64_t chi_l, int64_t chi_r,
                                              int32_t d, int32_t w, int32_t nv, itn_prec prec,
                                              size_t* bytes) {
  if (!h || !bytes) return ITN_E_ARG;
  if (!valid_prec(prec) || chi_l < 0 || chi_r < 0 || d < 1 || w < 1 || nv < 1)
    return fail(h, ITN_E_ARG, "bad arguments");
  *bytes = heff_ws_bytes(chi_l, chi_r, d, w, nv, prec, false, false);
  return ITN_OK;
}

// Shapes of one term of H_eff: L [chi_l, w, chi_l], R [chi_r, w, chi_r], W1 and
// W2 [w, w, d, d] host F64, against psi [chi_l, d, d, chi_r].
static itn_status check_term(itn_handle* h, const itn_tensor* L, const itn_tensor* W1,
                             const itn_tensor* W2, const itn_tensor* R, const itn_tensor* psi) {
  ITN_TRY(check_dense(h, L, "L", 3));
  ITN_TRY(check_dense(h, R, "R", 3));
  ITN_TRY(check_dense(h, W1, "W1", 4));
  ITN_TRY(check_dense(h, W2, "W2", 4));
  const int64_t cl = psi->dims[0], cr = psi->dims[3], d = psi->dims[1], w = L->dims[1];
  if (L->dims[0] != cl || L->dims[2] != cl) return fail(h, ITN_E_SHAPE, "L must be [chi_l, w, chi_l]");
  if (R->dims[0] != cr || R->dims[1] != w || R->dims[2] != cr)
    return fail(h, ITN_E_SHAPE, "R must be [chi_r, w, chi_r]");
  for (const itn_tensor* W : {W1, W2})
    if (W->dims[0] != w || W->dims[1] != w || W->dims[2] != d || W->dims[3] != d)
      return fail(h, ITN_E_SHAPE, "W must be [w, w, d, d] with w = %lld, d = %lld", (long long)w,
                  (long long)d);
  if (W1->dtype != ITN_F64 || W2->dtype != ITN_F64 || !W1->data || !W2->data)
    return fail(h, ITN_E_DTYPE, "W1, W2 must be host F64 arrays");
  return ITN_OK;
}

// Device bytes of a W-stage table held in a fixed scratch region.
static size_t table_bytes(const CSR& c) {
  const size_t nz = std::max<size_t>(1, c.coef.size());
  return round256(c.row_ptr.size() * 4) + round256(std::max<size_t>(1, c.row_off.size()) * 8) +
         round256(nz * 8) * 2 + round256(nz * 4) * 2;
}

// Copy a W-stage table into a fixed scratch region (stream-ordered before the
// kernels that read it); the returned WTable points into the region.
static itn_status table_to_scratch(itn_handle* h, const CSR& c, Carver& cv, hipStream_t s, WTable* t) {
  const size_t nz = std::max<size_t>(1, c.coef.size());
  t->nrows = (int32_t)c.row_off.size();
  t->nnz = (int64_t)c.coef.size();
  t->row_ptr = static_cast<int32_t*>(cv.take(c.row_ptr.size() * 4));
  t->row_off = static_cast<int64_t*>(cv.take(std::max<size_t>(1, c.row_off.size()) * 8));
  t->col_off = static_cast<int64_t*>(cv.take(nz * 8));
  t->coef = static_cast<double*>(cv.take(nz * 8));
  t->col_idx = static_cast<int32_t*>(cv.take(nz * 4));
  t->coef32 = static_cast<float*>(cv.take(nz * 4));
  ITN_HIP(h, hipMemcpyAsync(t->row_ptr, c.row_ptr.data(), c.row_ptr.size() * 4, hipMemcpyHostToDevice, s));
  if (!c.row_off.empty())
    ITN_HIP(h, hipMemcpyAsync(t->row_off, c.row_off.data(), c.row_off.size() * 8, hipMemcpyHostToDevice, s));
  if (!c.coef.empty()) {
    std::vector<int32_t> ci(c.col_off.begin(), c.col_off.end());
    std::vector<float> cf(c.coef.begin(), c.coef.end());
    ITN_HIP(h, hipMemcpyAsync(t->col_off, c.col_off.data(), c.col_off.size() * 8, hipMemcpyHostToDevice, s));
    ITN_HIP(h, hipMemcpyAsync(t->coef, c.coef.data(), c.coef.size() * 8, hipMemcpyHostToDevice, s));
    ITN_HIP(h, hipMemcpyAsync(t->col_idx, ci.data(), ci.size() * 4, hipMemcpyHostToDevice, s));
    ITN_HIP(h, hipMemcpyAsync(t->coef32, cf.data(), cf.size() * 4, hipMemcpyHostToDevice, s));
  }
  return ITN_OK;
}

namespace itn {

// out = sum over the n terms of H_eff,k psi (Sec. 7.2 sums of MPOs).  psi is
// transposed and cast once; every term runs stage 1 (+ W-stage) and its
// stage-4 GEMM adds into out from the second term on.  Scratch comes from the
// handle's workspace (grown on demand) with W-stage tables from the handle's
// content-keyed cache, or, when `fixed` is given, from that region alone
// (tables copied into it on the stream; nothing is allocated).
itn_status heff_apply_terms(itn_handle* h, int n, const itn_tensor* const* Ls,
                            const itn_tensor* const* W1s, const itn_tensor* const* W2s,
                            const itn_tensor* const* Rs, const itn_tensor* psi, int32_t nv,
                            itn_tensor* out, itn_prec prec, void* hip_stream,
                            const FixedScratch* fixed) {
  if (!h) return ITN_E_ARG;
  if (n < 1 || !Ls || !W1s || !W2s || !Rs) return fail(h, ITN_E_ARG, "need at least one term");
  ITN_TRY(check_dense(h, psi, "psi", 4));
  ITN_TRY(check_dense(h, out, "out", 4));
  if (!valid_prec(prec)) return fail(h, ITN_E_ARG, "unknown precision");
  if (nv < 1) return fail(h, ITN_E_ARG, "nv must be >= 1");
  if (psi->dims[1] != psi->dims[2]) return fail(h, ITN_E_SHAPE, "psi must be [chi_l, d, d, chi_r]");
  for (int k = 0; k < n; ++k) ITN_TRY(check_term(h, Ls[k], W1s[k], W2s[k], Rs[k], psi));
  const int64_t cl = psi->dims[0], cr = psi->dims[3];
  const int64_t d = psi->dims[1];
  for (int k = 0; k < 4; ++k)
    if (out->dims[k] != psi->dims[k]) return fail(h, ITN_E_SHAPE, "out must have psi's shape");
  if (psi->dtype == ITN_BF16 || out->dtype == ITN_BF16)
    return fail(h, ITN_E_DTYPE, "psi and out must be F64 or F32");
  if (h->device < 0 && !h->ws.query) return fail(h, ITN_E_NODEVICE, "host-only handle cannot launch work");
  const int64_t d2 = d * d;
  const int64_t n1 = cl * d2 * cr;  // one vector
  if (n1 == 0) return ITN_OK;
  if (!h->ws.query && (!psi->data || !out->data)) return fail(h, ITN_E_ARG, "psi and out need data");
  if (!h->ws.query) {  // the nv vectors of psi and of out occupy disjoint byte ranges
    const uintptr_t pa = reinterpret_cast<uintptr_t>(psi->data);
    const uintptr_t pb = reinterpret_cast<uintptr_t>(out->data);
    const uintptr_t na = (uintptr_t)(nv * n1) * dtype_size(psi->dtype);
    const uintptr_t nb = (uintptr_t)(nv * n1) * dtype_size(out->dtype);
    if (pa < pb + nb && pb < pa + na) return fail(h, ITN_E_ARG, "out must not overlap psi");
  }
  hipStream_t s = as_stream(hip_stream);
  const int P = prec;
  const int pt = P == ITN_P_F64 ? D_F64 : (P == ITN_P_F32 ? D_F32 : D_BF16);
  const int es = dtype_size(pt);
  const int xt = xtype_of(P);
  const int64_t N1 = d2 * nv * cr;
  int64_t wmax = 0, wmax_unfused = 0;
  bool anyL = false, anyR = false;
  // Per term: fused stage 1 or not, and the W-stage table it reads.
  //   fused:   CSR with input index m0*d2 + c and output row c'*w + m2
  //   unfused: CSR over X[a'][m0][c][v][b] -> Z[v][a'][c'][m2][b]
  std::vector<char> fused(n, 0);
  std::vector<CSR> csrs(n);
  // The fused stage-1 kernel loads L rows straight into LDS: whole 128-byte
  // K steps and 16-byte aligned rows (a converted L lands in aligned scratch).
  const int64_t bk = 128 / es;
  for (int k = 0; k < n; ++k) {
    const int64_t w = Ls[k]->dims[1];
    wmax = std::max(wmax, w);
    anyL |= Ls[k]->dtype != pt;
    anyR |= Rs[k]->dtype != pt;
    const double* w1 = static_cast<const double*>(W1s[k]->data);
    const double* w2 = static_cast<const double*>(W2s[k]->data);
    const bool aligned = Ls[k]->dtype != pt || (reinterpret_cast<uintptr_t>(Ls[k]->data) & 15) == 0;
    bool f = heff_fused_supported(P, (int)w, (int)d2) && cl % bk == 0 && cl > 0 && aligned &&
             heff_fused_fits(P, cl, cr, (int)w, (int)d2, (int)nv);
    if (f) {
      csrs[k] = heff_w_csr(w1, w2, (int)w, (int)d, d2, 1, w, 1);
      f = heff_fused_table_fits((int)csrs[k].row_off.size(), (int64_t)csrs[k].coef.size());
    }
    if (!f) {
      csrs[k] = heff_w_csr(w1, w2, (int)w, (int)d, /*in_m*/ N1, /*in_c*/ (int64_t)nv * cr,
                           /*out_c*/ w * cr, /*out_m*/ cr);
      wmax_unfused = std::max(wmax_unfused, w);
    }
    fused[k] = f;
  }
  const size_t bLc = anyL ? round256((size_t)(cl * wmax * cl) * es) : 0;
  const size_t bRc = anyR ? round256((size_t)(cr * wmax * cr) * es) : 0;
  const size_t bPT = round256((size_t)(d2 * nv * cr * cl) * es);
  const size_t bZ = round256((size_t)(nv * cl * d2 * wmax * cr) * es);
  const size_t bX = round256((size_t)(cl * wmax_unfused * d2 * nv * cr) * dtype_size(xt));
  size_t need = bLc + bRc + bPT + bZ + bX;
  void* base = nullptr;
  if (fixed) {
    for (int k = 0; k < n; ++k) need += table_bytes(csrs[k]);
    if (need > fixed->bytes)
      return fail(h, ITN_E_WORKSPACE,
                  "this H_eff needs %zu bytes of scratch; the fixed scratch region holds %zu", need,
                  fixed->bytes);
    base = fixed->base;
  } else {
    ITN_TRY(ensure_workspace(h, need + 256));
    base = h->ws.ptr;
  }
  Carver cv(base);
  void* Lcast = anyL ? cv.take(bLc) : nullptr;
  void* Rcast = anyR ? cv.take(bRc) : nullptr;
  void* psiT = cv.take(bPT);
  void* Z = cv.take(bZ);
  void* Xbuf = bX ? cv.take(bX) : nullptr;
  std::vector<WTable> fixed_tabs(fixed ? n : 0);
  if (fixed)
    for (int k = 0; k < n; ++k) ITN_TRY(table_to_scratch(h, csrs[k], cv, s, &fixed_tabs[k]));
  // psi[v][a][c][b] -> psiT[c][v][b][a]
  TransposeArgs ta{};
  ta.rows = cl;
  ta.cols = cr;
  ta.nzb = nv;
  ta.nzc = d2;
  ta.in_zb = n1;
  ta.in_zc = cr;
  ta.in_r = d2 * cr;
  ta.in_c = 1;
  ta.out_zb = cr * cl;
  ta.out_zc = (int64_t)nv * cr * cl;
  ta.out_c = cl;
  ta.out_r = 1;
  {
    Prof pf(h, "heff_psi_transpose", s);
    ITN_HIP(h, transpose_cast(psi->dtype, psi->data, pt, psiT, ta, s));
  }
  for (int term = 0; term < n; ++term) {
    const itn_tensor* L = Ls[term];
    const itn_tensor* R = Rs[term];
    const int64_t w = L->dims[1];
    const void* Lp = L->data;
    const void* Rp = R->data;
    if (L->dtype != pt) {
      Prof pf(h, "cast_env", s);
      ITN_HIP(h, cast(L->dtype, L->data, pt, Lcast, cl * w * cl, s));
      Lp = Lcast;
    }
    if (R->dtype != pt) {
      Prof pf(h, "cast_env", s);
      ITN_HIP(h, cast(R->dtype, R->data, pt, Rcast, cr * w * cr, s));
      Rp = Rcast;
    }
    const CSR& csr = csrs[term];
    const WTable* tab = nullptr;
    if (fixed) tab = &fixed_tabs[term];
    else
      ITN_TRY(get_wtable(h, (fused[term] ? "fused" : "") + csr.key(), csr.row_ptr, csr.row_off,
                         csr.col_off, csr.coef, &tab));
    if (fused[term]) {
      HeffFusedArgs fa{};
      fa.L = Lp;
      fa.psiT = psiT;
      fa.Z = Z;
      fa.chi_l = cl;
      fa.chi_r = cr;
      fa.w = (int)w;
      fa.d2 = (int)d2;
      fa.nv = nv;
      fa.nrows = tab->nrows;
      fa.nnz = (int32_t)tab->nnz;
      fa.row_ptr = tab->row_ptr;
      fa.col_idx = tab->col_idx;
      fa.coef32 = tab->coef32;
      fa.coef64 = tab->coef;
      Prof pf(h, "heff_stage1_fused", s);
      ITN_HIP(h, heff_stage1_fused(P, fa, s));
    } else {
      // Stage 1: X[(a' m0), (c v b)] = L[(a' m0), a] . psiT[(c v b), a]
      GemmArgs g1{};
      g1.A = Lp;
      g1.B = psiT;
      g1.C = Xbuf;
      g1.M = cl * w;
      g1.N = N1;
      g1.K = cl;
      g1.lda = cl;
      g1.ldb = cl;
      g1.ldc = N1;
      g1.batch = 1;
      {
        Prof pf(h, "heff_stage1_gemm", s);
        ITN_HIP(h, gemm_nt(P, xt, g1, s));
      }
      // W-stage: Z[v][a'][c'][m2][b] = sum W12 X[a'][m0][c][v][b]
      WStageArgs wa{};
      wa.X = cl;
      wa.Z = nv;
      wa.Y = cr;
      wa.isx = w * N1;
      wa.isz = cr;
      wa.isy = 1;
      wa.osx = d2 * w * cr;
      wa.osz = cl * d2 * w * cr;
      wa.osy = 1;
      wa.nrows = tab->nrows;
      Prof pf(h, "heff_wstage", s);
      ITN_HIP(h, wstage(xt, Xbuf, pt, Z, wa, tab->row_ptr, tab->row_off, tab->col_off, tab->coef, s));
    }
    // Stage 4: out[(v a' c'), b'] (+)= Z[(v a' c'), (m2 b)] . R[b', (m2 b)]
    GemmArgs g4{};
    g4.A = Z;
    g4.B = Rp;
    g4.C = out->data;
    g4.M = (int64_t)nv * cl * d2;
    g4.N = cr;
    g4.K = w * cr;
    g4.lda = w * cr;
    g4.ldb = w * cr;
    g4.ldc = cr;
    g4.batch = 1;
    g4.accumulate = term > 0;
    g4.stream = 1;  // H psi is read by the eigensolver's next pass, not by a resident kernel
    Prof pf(h, "heff_stage4_gemm", s);
    ITN_HIP(h, gemm_nt(P, out->dtype, g4, s));
  }
  return ITN_OK;
}

}  // namespace itn

extern "C" {

itn_status itn_set_workspace(itn_handle* h, void* ptr, size_t bytes) {
  if (!h) return ITN_E_ARG;
  if (h->device < 0) return fail(h, ITN_E_NODEVICE, "host-only handle has no workspace");
  if (ptr && (reinterpret_cast<uintptr_t>(ptr) & 255) != 0)
    return fail(h, ITN_E_ARG, "workspace must be 256-byte aligned");
  if (!ptr && bytes != 0) return fail(h, ITN_E_ARG, "NULL workspace with a nonzero size");
  ITN_HIP(h, hipDeviceSynchronize());
  if (h->ws.ptr && !h->ws.caller) ITN_HIP(h, hipFree(h->ws.ptr));
  h->ws.ptr = ptr;
  h->ws.size = ptr ? bytes : 0;
  h->ws.caller = ptr != nullptr;
  return ITN_OK;
}

itn_status itn_workspace_size(itn_handle* h, itn_op op, int32_t ntensors, const itn_tensor* const* t,
                              int32_t nv, int32_t dir, itn_prec prec, size_t* bytes) {
  if (!h || !bytes || (ntensors > 0 && !t)) return h ? fail(h, ITN_E_ARG, "null argument") : ITN_E_ARG;
  const int need = op == ITN_OP_CONTRACT ? 3 : op == ITN_OP_HEFF ? 5 : op == ITN_OP_ENV_UPDATE ? 4 : -1;
  if (need < 0) return fail(h, ITN_E_ARG, "unknown operation");
  if (ntensors != need) return fail(h, ITN_E_ARG, "this operation takes %d tensors", need);
  // The call itself, stopped at its workspace request (validation included).
  h->ws.query = true;
  h->ws.query_bytes = 0;
  itn_status st = ITN_OK;
  if (op == ITN_OP_CONTRACT)
    st = itn_contract(h, t[0], t[1], const_cast<itn_tensor*>(t[2]), prec, nullptr);
  else if (op == ITN_OP_HEFF)
    st = heff_apply_terms(h, 1, &t[0], &t[1], &t[2], &t[3], t[4], nv, const_cast<itn_tensor*>(t[4]),
                          prec, nullptr, nullptr);
  else
    st = itn_env_update(h, t[0], t[1], t[2], (itn_dir)dir, const_cast<itn_tensor*>(t[3]), prec, nullptr);
  h->ws.query = false;
  if (st == ITN_STOP_QUERY || st == ITN_OK) {
    *bytes = st == ITN_OK ? 0 : h->ws.query_bytes;
    return ITN_OK;
  }
  return st;
}

itn_status itn_heff_apply(itn_handle* h, const itn_tensor* L, const itn_tensor* W1,
                          const itn_tensor* W2, const itn_tensor* R, const itn_tensor* psi,
                          int32_t nv, itn_tensor* out, itn_prec prec, void* hip_stream) {
  return heff_apply_terms(h, 1, &L, &W1, &W2, &R, psi, nv, out, prec, hip_stream, nullptr);
}

itn_status itn_heff_apply_sum(itn_handle* h, int32_t nterms, const itn_tensor* const* L,
                              const itn_tensor* const* W1, const itn_tensor* const* W2,
                              const itn_tensor* const* R, const itn_tensor* psi, int32_t nv,
                              itn_tensor* out, itn_prec prec, void* hip_stream) {
  return heff_apply_terms(h, nterms, L, W1, W2, R, psi, nv, out, prec, hip_stream, nullptr);
}

// --------------------------------------------------------- environment step
itn_status itn_env_update(itn_handle* h, const itn_tensor* E, const itn_tensor* A,
                          const itn_tensor* W, itn_dir dir, itn_tensor* E_out, itn_prec prec,
                          void* hip_stream) {
  if (!h) return ITN_E_ARG;
  ITN_TRY(check_dense(h, E, "E", 3));
  ITN_TRY(check_dense(h, A, "A", 3));
  ITN_TRY(check_dense(h, W, "W", 4));
  ITN_TRY(check_dense(h, E_out, "E_out", 3));
  if (!valid_prec(prec)) return fail(h, ITN_E_ARG, "unknown precision");
  if (dir != ITN_LEFT && dir != ITN_RIGHT) return fail(h, ITN_E_ARG, "dir must be ITN_LEFT or ITN_RIGHT");
  if (W->dtype != ITN_F64 || !W->data) return fail(h, ITN_E_DTYPE, "W must be a host F64 array");
  if (E->dtype == ITN_BF16 || A->dtype == ITN_BF16 || E_out->dtype == ITN_BF16)
    return fail(h, ITN_E_DTYPE, "E, A, E_out must be F64 or F32");
  const int64_t w = E->dims[1], d = A->dims[1];
  if (W->dims[0] != w || W->dims[1] != w || W->dims[2] != d || W->dims[3] != d)
    return fail(h, ITN_E_SHAPE, "W must be [w, w, d, d]");
  if (E->dims[0] != E->dims[2]) return fail(h, ITN_E_SHAPE, "E must be [chi, w, chi]");
  const int64_t chi = E->dims[0];
  const int64_t chio = dir == ITN_LEFT ? A->dims[2] : A->dims[0];
  const int64_t chii = dir == ITN_LEFT ? A->dims[0] : A->dims[2];
  if (chii != chi) return fail(h, ITN_E_SHAPE, "A's %s bond (%lld) must match E (%lld)",
                               dir == ITN_LEFT ? "left" : "right", (long long)chii, (long long)chi);
  if (E_out->dims[0] != chio || E_out->dims[1] != w || E_out->dims[2] != chio)
    return fail(h, ITN_E_SHAPE, "E_out must be [%lld, %lld, %lld]", (long long)chio, (long long)w,
                (long long)chio);
  if (h->device < 0 && !h->ws.query) return fail(h, ITN_E_NODEVICE, "host-only handle cannot launch work");
  hipStream_t s = as_stream(hip_stream);
  if (chio == 0) return ITN_OK;
  const int P = prec;
  const int pt = P == ITN_P_F64 ? D_F64 : (P == ITN_P_F32 ? D_F32 : D_BF16);
  const int es = dtype_size(pt);
  const int xt = xtype_of(P);
  const int xs = dtype_size(xt);
  const double* Wh = static_cast<const double*>(W->data);
  if (chi == 0) {
    ITN_HIP(h, fill(E_out->data, E_out->dtype, 0.0, chio * w * chio, s));
    return ITN_OK;
  }
  const size_t bE = round256((size_t)(chi * w * chi) * es);
  const size_t bA = round256((size_t)(chi * d * chio) * es);
  const size_t bT = round256((size_t)(chi * w * d * chio) * xs);
  const size_t bT2 = round256((size_t)(chi * w * d * chio) * es);
  ITN_TRY(ensure_workspace(h, bE + 2 * bA + bT + bT2 + 256));
  Carver cv(h->ws.ptr);
  const void* Ep = E->data;
  if (E->dtype != pt) {
    void* t = cv.take(bE);
    ITN_HIP(h, cast(E->dtype, E->data, pt, t, chi * w * chi, s));
    Ep = t;
  }
  void* T1 = cv.take(bT);
  void* T2 = cv.take(bT2);
  if (dir == ITN_LEFT) {
    // A[a''' or a''][s][a] : chi x d x chio
    void* AT = cv.take(bA);   // [s][a][a''']
    void* AT2 = cv.take(bA);  // [a'][(a'' s')]
    TransposeArgs t1{};
    t1.rows = chi;
    t1.cols = chio;
    t1.nzb = 1;
    t1.nzc = d;
    t1.in_zc = chio;
    t1.in_r = d * chio;
    t1.in_c = 1;
    t1.out_zc = chio * chi;
    t1.out_c = chi;
    t1.out_r = 1;
    ITN_HIP(h, transpose_cast(A->dtype, A->data, pt, AT, t1, s));
    TransposeArgs t2{};
    t2.rows = chi * d;
    t2.cols = chio;
    t2.nzb = 1;
    t2.nzc = 1;
    t2.in_r = chio;
    t2.in_c = 1;
    t2.out_c = chi * d;
    t2.out_r = 1;
    ITN_HIP(h, transpose_cast(A->dtype, A->data, pt, AT2, t2, s));
    // T1[(s a), (a'' m)] = AT[(s a), a'''] . E[(a'' m), a''']
    GemmArgs g{};
    g.A = AT;
    g.B = Ep;
    g.C = T1;
    g.M = d * chio;
    g.N = chi * w;
    g.K = chi;
    g.lda = chi;
    g.ldb = chi;
    g.ldc = chi * w;
    g.batch = 1;
    ITN_HIP(h, gemm_nt(P, xt, g, s));
    // T2[m'][a][a''][s'] = sum_{m,s} W[m,m',s',s] T1[s][a][a''][m]
    CSR csr = env_w_csr(Wh, (int)w, (int)d, true, /*in_m*/ 1, /*in_s*/ chio * chi * w,
                        /*out_m*/ chio * chi * d, /*out_s*/ 1);
    const WTable* tab = nullptr;
    ITN_TRY(get_wtable(h, csr.key(), csr.row_ptr, csr.row_off, csr.col_off, csr.coef, &tab));
    WStageArgs wa{};
    wa.X = chio;
    wa.Z = 1;
    wa.Y = chi;
    wa.isx = chi * w;
    wa.isy = w;
    wa.osx = chi * d;
    wa.osy = d;
    wa.nrows = tab->nrows;
    ITN_HIP(h, wstage(xt, T1, pt, T2, wa, tab->row_ptr, tab->row_off, tab->col_off, tab->coef, s));
    // E_out[a', (m' a)] = AT2[a', (a'' s')] . T2[(m' a), (a'' s')]
    GemmArgs g2{};
    g2.A = AT2;
    g2.B = T2;
    g2.C = E_out->data;
    g2.M = chio;
    g2.N = w * chio;
    g2.K = chi * d;
    g2.lda = chi * d;
    g2.ldb = chi * d;
    g2.ldc = w * chio;
    g2.batch = 1;
    ITN_HIP(h, gemm_nt(P, E_out->dtype, g2, s));
  } else {
    // A[b][s][b'''] : chio x d x chi
    const void* Ap = A->data;
    if (A->dtype != pt) {
      void* t = cv.take(bA);
      ITN_HIP(h, cast(A->dtype, A->data, pt, t, chio * d * chi, s));
      Ap = t;
    }
    // T1[(b s), (b'' m')] = A[(b s), b'''] . E[(b'' m'), b''']
    GemmArgs g{};
    g.A = Ap;
    g.B = Ep;
    g.C = T1;
    g.M = chio * d;
    g.N = chi * w;
    g.K = chi;
    g.lda = chi;
    g.ldb = chi;
    g.ldc = chi * w;
    g.batch = 1;
    ITN_HIP(h, gemm_nt(P, xt, g, s));
    // T2[m][b][s'][b''] = sum_{m',s} W[m,m',s',s] T1[b][s][b''][m']
    CSR csr = env_w_csr(Wh, (int)w, (int)d, false, /*in_m*/ 1, /*in_s*/ chi * w,
                        /*out_m*/ chio * d * chi, /*out_s*/ chi);
    const WTable* tab = nullptr;
    ITN_TRY(get_wtable(h, csr.key(), csr.row_ptr, csr.row_off, csr.col_off, csr.coef, &tab));
    WStageArgs wa{};
    wa.X = chio;
    wa.Z = 1;
    wa.Y = chi;
    wa.isx = d * chi * w;
    wa.isy = w;
    wa.osx = d * chi;
    wa.osy = 1;
    wa.nrows = tab->nrows;
    ITN_HIP(h, wstage(xt, T1, pt, T2, wa, tab->row_ptr, tab->row_off, tab->col_off, tab->coef, s));
    // E_out[b', (m b)] = A[b', (s' b'')] . T2[(m b), (s' b'')]
    GemmArgs g2{};
    g2.A = Ap;
    g2.B = T2;
    g2.C = E_out->data;
    g2.M = chio;
    g2.N = w * chio;
    g2.K = d * chi;
    g2.lda = d * chi;
    g2.ldb = d * chi;
    g2.ldc = w * chio;
    g2.batch = 1;
    ITN_HIP(h, gemm_nt(P, E_out->dtype, g2, s));
  }
  return ITN_OK;
}

}  // extern "C"
