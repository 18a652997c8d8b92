// Quantum-number bookkeeping shared by the block-sparse calls (host side):
// QN indices and tensors as the ABI describes them (Sec. 8: sectors, arrows,
// flux; Sec. 9.2: blocks at offsets in one array), read and validated.
#pragma once

#include <algorithm>
#include <functional>
#include <map>
#include <vector>

#include "handle.h"

namespace itn {
namespace qn {

// QN component c adds modulo mod[c] when mod[c] > 0 (Z_N), else as integers.
inline int32_t qn_red(int64_t x, int32_t m) { return m > 0 ? (int32_t)(((x % m) + m) % m) : (int32_t)x; }

struct QSpace {
  int nsec = 0, nq = 0;
  std::vector<int32_t> qn;   // nsec*nq, Z_N components reduced into [0, N)
  std::vector<int32_t> mod;  // nq addition rules (0 = integer)
  std::vector<int32_t> dim;  // nsec
  std::vector<int64_t> off;  // element offset of each sector
  int8_t arrow = 0;
  int64_t total = 0;
  const int32_t* q(int k) const { return qn.data() + (size_t)k * nq; }
  bool same_sectors(const QSpace& o) const {
    return nq == o.nq && qn == o.qn && dim == o.dim && mod == o.mod;
  }
  // sector with exactly this QN, or -1 (sectors with distinct QNs only)
  int find(const std::vector<int32_t>& want) const {
    for (int k = 0; k < nsec; ++k)
      if (std::equal(want.begin(), want.end(), q(k))) return k;
    return -1;
  }
};

struct QTensor {
  int rank = 0;
  std::vector<QSpace> sp;
  std::vector<std::vector<int32_t>> blocks;  // sector tuples
  std::vector<int64_t> off;
  std::map<std::vector<int32_t>, int> index;
  int64_t elems = 0;
};

inline itn_status read_space(itn_handle* h, const itn_space& s, QSpace& out, const char* what) {
  if (s.nsec < 1 || s.nq < 1 || !s.qn || !s.dim)
    return fail(h, ITN_E_ARG, "%s: a QN index needs nsec >= 1, nq >= 1, qn and dim", what);
  if (s.arrow != 1 && s.arrow != -1) return fail(h, ITN_E_ARROW, "%s: arrow must be +1 or -1", what);
  out.nsec = s.nsec;
  out.nq = s.nq;
  out.mod.assign(s.nq, 0);
  if (s.mod) {
    for (int c = 0; c < s.nq; ++c) {
      if (s.mod[c] < 0 || s.mod[c] == 1)
        return fail(h, ITN_E_ARG, "%s: a QN addition rule is 0 (integer) or N >= 2 (Z_N)", what);
      out.mod[c] = s.mod[c];
    }
  }
  out.qn.assign(s.qn, s.qn + (size_t)s.nsec * s.nq);
  for (size_t k = 0; k < out.qn.size(); ++k) out.qn[k] = qn_red(out.qn[k], out.mod[k % s.nq]);
  out.dim.assign(s.dim, s.dim + s.nsec);
  out.arrow = s.arrow;
  out.off.resize(s.nsec);
  out.total = 0;
  for (int k = 0; k < s.nsec; ++k) {
    if (out.dim[k] < 1) return fail(h, ITN_E_SHAPE, "%s: sector dimensions must be >= 1", what);
    out.off[k] = out.total;
    out.total += out.dim[k];
  }
  return ITN_OK;
}

inline std::vector<int32_t> block_flux(const QTensor& t, const std::vector<int32_t>& blk) {
  const int nq = t.sp[0].nq;
  std::vector<int64_t> f(nq, 0);
  for (int i = 0; i < t.rank; ++i)
    for (int c = 0; c < nq; ++c) f[c] += t.sp[i].arrow * t.sp[i].q(blk[i])[c];
  std::vector<int32_t> r(nq);
  for (int c = 0; c < nq; ++c) r[c] = qn_red(f[c], t.sp[0].mod[c]);
  return r;
}

// a + sb * b under the QN addition rules `mod`.
inline std::vector<int32_t> qadd(const int32_t* a, const int32_t* b, const std::vector<int32_t>& mod, int sb) {
  const int nq = (int)mod.size();
  std::vector<int32_t> r(nq);
  for (int c = 0; c < nq; ++c) r[c] = qn_red((int64_t)a[c] + sb * (int64_t)b[c], mod[c]);
  return r;
}

// Every allowed sector tuple of a tensor's indices (flux `flux`, empty =
// zero), lexicographic.
inline std::vector<std::vector<int32_t>> allowed_blocks(const QTensor& t,
                                                       const std::vector<int32_t>& flux = {}) {
  std::vector<std::vector<int32_t>> out;
  std::vector<int32_t> blk(t.rank, 0);
  const int nq = t.sp[0].nq;
  std::function<void(int)> rec = [&](int i) {
    if (i == t.rank) {
      auto f = block_flux(t, blk);
      bool zero = true;
      for (int c = 0; c < nq; ++c) zero &= f[c] == (flux.empty() ? 0 : flux[c]);
      if (zero) out.push_back(blk);
      return;
    }
    for (int k = 0; k < t.sp[i].nsec; ++k) {
      blk[i] = k;
      rec(i + 1);
    }
  };
  rec(0);
  return out;
}

// Diagonal of the two-site block-sparse H_eff (the block Davidson
// preconditioner), psi's block layout.  An entry pairs L[a, m0, a] with
// R[b, m2, b]: the environments' flux rule leaves only their blocks whose two
// link sectors coincide, all on zero-charge MPO channels, whose diagonals
// are gathered into dense [chi][zero-charge channels] tables; Wd[i][j][s1][s2]
// = sum_m1 W1[m0, m1, s1, s1] W2[m1, m2, s2, s2] over those channels.
// heff_diag_build lays out the host tables (integer and FP64 host work);
// heff_diag_launch uploads them to `dev` (device_bytes() of device memory,
// 256-byte aligned) on stream s and launches; the host tables must stay alive
// until the stream has passed the upload.
struct HeffDiag {
  std::vector<char> host;  // Wd, the two environment item lists, psi's block list
  size_t o_li = 0, o_ri = 0, o_db = 0;
  int nli = 0, nri = 0, ndb = 0, wzl = 1, wzr = 1, d1 = 0, d2 = 0;
  int64_t cl = 0, cr = 0, most = 0;
  size_t device_bytes() const { return round256(host.size()) + (size_t)(cl * wzl + cr * wzr) * 8; }
};
// W1 [wl][wm][d1][d1], W2 [wm][wr][d2][d2] host FP64 (wl = L's channel total,
// wr = R's); L [a', m0, a], R [b', m2, b], P [a, s1, s2, b] structures.
itn_status heff_diag_build(itn_handle* h, const QTensor& L, const QTensor& R, const double* W1,
                           const double* W2, int wm, const QTensor& P, HeffDiag& out);
hipError_t heff_diag_launch(const HeffDiag& q, const double* Ldata, const double* Rdata, void* dev, double* D,
                            hipStream_t s);

}  // namespace qn
}  // namespace itn
