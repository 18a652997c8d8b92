// Labelled contraction of block-sparse (QN) tensors, the itn_contract path
// for operands that carry QN index spaces.
//
// Sec. 9.4 computes a block-sparse contraction as dense contractions of the
// block pairs whose contracted sectors agree, several pairs possibly landing
// on one output block; Sec. 8 fixes the rules checked here: contracted
// indices need opposite arrows, blocks obey their tensor's flux rule, and
// the flux of the product is the sum of the fluxes.  On the GPU every block
// of A and B is permuted once into a K-contiguous matrix, and all block
// products run as one grouped GEMM launch: one problem per output block,
// whose K is the concatenation of its contributing pairs in ascending pair
// order, summed by the workgroup that owns each output tile.
#include <cstring>
#include <set>

#include "handle.h"
#include "qn_common.h"

using namespace itn;
using namespace itn::qn;

namespace {

// Read a QN tensor with any arrows and flux t->flux (NULL = zero); blocks
// sorted, unique, flux-allowed, offsets the exclusive prefix sum.
itn_status read_qn_any(itn_handle* h, const itn_tensor* t, QTensor& out, std::vector<int32_t>& flux,
                       const char* what) {
  if (!t) return fail(h, ITN_E_ARG, "%s is NULL", what);
  if (t->rank < 0 || t->rank > 8) return fail(h, ITN_E_SHAPE, "%s rank %d out of range", what, t->rank);
  if (t->rank > 0 && !t->space) return fail(h, ITN_E_ARG, "%s needs QN index spaces", what);
  out.rank = t->rank;
  out.sp.resize(t->rank);
  for (int i = 0; i < t->rank; ++i) {
    ITN_TRY(read_space(h, t->space[i], out.sp[i], what));
    if (out.sp[i].nq != out.sp[0].nq) return fail(h, ITN_E_SHAPE, "%s: mixed QN lengths", what);
    if (out.sp[i].mod != out.sp[0].mod) return fail(h, ITN_E_SHAPE, "%s: mixed QN addition rules", what);
  }
  if (t->nblocks < 0 || (t->nblocks > 0 && (!t->block_off || (t->rank > 0 && !t->block_sec))))
    return fail(h, ITN_E_ARG, "%s: block list missing", what);
  const int nq = t->rank > 0 ? out.sp[0].nq : 0;
  flux.assign(nq, 0);
  if (t->flux && nq > 0) {
    for (int c = 0; c < nq; ++c) flux[c] = qn_red(t->flux[c], out.sp[0].mod[c]);
  }
  int64_t expect = 0;
  for (int64_t b = 0; b < t->nblocks; ++b) {
    std::vector<int32_t> blk(t->rank);
    for (int i = 0; i < t->rank; ++i) blk[i] = t->block_sec[b * t->rank + i];
    int64_t sz = 1;
    for (int i = 0; i < t->rank; ++i) {
      if (blk[i] < 0 || blk[i] >= out.sp[i].nsec)
        return fail(h, ITN_E_ARG, "%s block %lld: sector out of range", what, (long long)b);
      sz *= out.sp[i].dim[blk[i]];
    }
    if (b > 0 && !(out.blocks.back() < blk)) return fail(h, ITN_E_ARG, "%s blocks must be sorted and unique", what);
    if (t->rank > 0 && block_flux(out, blk) != flux)
      return fail(h, ITN_E_FLUX, "%s block %lld violates the flux rule", what, (long long)b);
    if (t->block_off[b] != expect)
      return fail(h, ITN_E_SHAPE, "%s block offsets must be the exclusive prefix sum of block sizes", what);
    expect += sz;
    out.index[blk] = (int)out.blocks.size();
    out.blocks.push_back(blk);
    out.off.push_back(t->block_off[b]);
  }
  out.elems = expect;
  return ITN_OK;
}

int find_label(const itn_tensor* t, int32_t l) {
  for (int k = 0; k < t->rank; ++k)
    if (t->label[k] == l) return k;
  return -1;
}

}  // namespace

namespace itn {

itn_status contract_qn(itn_handle* h, const itn_tensor* A, const itn_tensor* B, itn_tensor* C,
                       itn_prec prec, void* hip_stream) {
  if (!A->space && A->rank > 0) return fail(h, ITN_E_ARG, "A is dense and B or C block-sparse: mix not supported");
  if (!B->space && B->rank > 0) return fail(h, ITN_E_ARG, "B is dense and A or C block-sparse: mix not supported");
  if (!C->space && C->rank > 0) return fail(h, ITN_E_ARG, "C must be block-sparse like A and B");
  if ((A->rank && !A->label) || (B->rank && !B->label) || (C->rank && !C->label))
    return fail(h, ITN_E_ARG, "labels missing");
  for (const itn_tensor* t : {A, B, static_cast<const itn_tensor*>(C)})
    if (t->dtype != ITN_F64 && t->dtype != ITN_F32)
      return fail(h, ITN_E_DTYPE, "block-sparse operands must be F64 or F32");
  QTensor qa, qb, qc;
  std::vector<int32_t> fa, fb, fc;
  ITN_TRY(read_qn_any(h, A, qa, fa, "A"));
  ITN_TRY(read_qn_any(h, B, qb, fb, "B"));
  ITN_TRY(read_qn_any(h, C, qc, fc, "C"));
  auto uniq = [](const itn_tensor* t) {
    std::set<int32_t> st(t->label, t->label + t->rank);
    return (int)st.size() == t->rank;
  };
  if (!uniq(A) || !uniq(B) || !uniq(C)) return fail(h, ITN_E_LABEL, "repeated label in an operand");
  // label roles
  std::vector<int> freeA, freeB, conA, conB;
  for (int k = 0; k < A->rank; ++k) {
    const int j = find_label(B, A->label[k]);
    if (j < 0) {
      freeA.push_back(k);
      continue;
    }
    const QSpace &ia = qa.sp[k], &ib = qb.sp[j];
    if (ia.arrow == ib.arrow)
      return fail(h, ITN_E_ARROW, "contracted label %d has equal arrows on A and B", A->label[k]);
    if (!ia.same_sectors(ib))
      return fail(h, ITN_E_SHAPE, "contracted label %d has different sectors on A and B", A->label[k]);
    conA.push_back(k);
    conB.push_back(j);
  }
  for (int k = 0; k < B->rank; ++k)
    if (find_label(A, B->label[k]) < 0) freeB.push_back(k);
  if ((int)(freeA.size() + freeB.size()) != C->rank)
    return fail(h, ITN_E_LABEL, "C must carry exactly the uncontracted labels");
  // C index k <- (operand, axis); its space must equal that index's
  std::vector<int> csrc(C->rank), cax(C->rank);
  for (int k = 0; k < C->rank; ++k) {
    const int ja = find_label(A, C->label[k]), jb = find_label(B, C->label[k]);
    const bool inA = ja >= 0 && jb < 0, inB = jb >= 0 && ja < 0;
    if (!inA && !inB) return fail(h, ITN_E_LABEL, "C label %d is not an uncontracted label", C->label[k]);
    const QSpace& src = inA ? qa.sp[ja] : qb.sp[jb];
    if (qc.sp[k].arrow != src.arrow)
      return fail(h, ITN_E_ARROW, "C label %d must keep its arrow", C->label[k]);
    if (!qc.sp[k].same_sectors(src))
      return fail(h, ITN_E_SHAPE, "C label %d must keep its sectors", C->label[k]);
    csrc[k] = inA ? 0 : 1;
    cax[k] = inA ? ja : jb;
  }
  // QN lengths and rules agree across the operands; flux(C) = flux(A) + flux(B)
  std::vector<int32_t> mod;
  int nq = -1;
  for (const QTensor* q : {&qa, &qb, &qc})
    if (q->rank > 0) {
      if (nq < 0) {
        nq = q->sp[0].nq;
        mod = q->sp[0].mod;
      } else if (q->sp[0].nq != nq || q->sp[0].mod != mod) {
        return fail(h, ITN_E_SHAPE, "operands use different QN lengths or addition rules");
      }
    }
  if (nq > 0) {
    auto pad = [&](std::vector<int32_t>& f) { if ((int)f.size() < nq) f.assign(nq, 0); };
    pad(fa);
    pad(fb);
    pad(fc);
    const auto want = qadd(fa.data(), fb.data(), mod, +1);
    if (want != fc) return fail(h, ITN_E_FLUX, "flux(C) must equal flux(A) + flux(B)");
  }
  if (prec != ITN_P_F64 && prec != ITN_P_F32 && prec != ITN_P_BF16)
    return fail(h, ITN_E_ARG, "unknown precision");
  // block pairs: B's blocks by their contracted-sector tuple (in A's con order)
  std::map<std::vector<int32_t>, std::vector<int>> bsec;
  for (size_t b = 0; b < qb.blocks.size(); ++b) {
    std::vector<int32_t> key;
    for (int j : conB) key.push_back(qb.blocks[b][j]);
    bsec[key].push_back((int)b);
  }
  struct Pair {
    int a, b;
  };
  std::map<int, std::vector<Pair>> by_c;  // C block -> pairs, ascending (a, b)
  for (size_t a = 0; a < qa.blocks.size(); ++a) {
    std::vector<int32_t> key;
    for (int k : conA) key.push_back(qa.blocks[a][k]);
    auto it = bsec.find(key);
    if (it == bsec.end()) continue;
    for (int b : it->second) {
      std::vector<int32_t> cblk(C->rank);
      for (int k = 0; k < C->rank; ++k)
        cblk[k] = csrc[k] == 0 ? qa.blocks[a][cax[k]] : qb.blocks[b][cax[k]];
      auto ci = qc.index.find(cblk);
      if (ci == qc.index.end())
        return fail(h, ITN_E_FLUX, "C lacks an output block that a contributing block pair reaches");
      by_c[ci->second].push_back(Pair{(int)a, b});
    }
  }
  if (h->device < 0 && !h->ws.query) return fail(h, ITN_E_NODEVICE, "host-only handle cannot launch work");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (qc.elems == 0) return ITN_OK;
  if (!h->ws.query && (!C->data || (qa.elems > 0 && !A->data) || (qb.elems > 0 && !B->data)))
    return fail(h, ITN_E_ARG, "operand data missing");
  const int P = prec;
  const int pt = P == ITN_P_F64 ? D_F64 : (P == ITN_P_F32 ? D_F32 : D_BF16);
  const int acc_dt = P == ITN_P_F64 ? D_F64 : D_F32;
  const int es = dtype_size(pt);
  // natural order of C: [free A..., free B...]
  bool natural = true;
  {
    int k = 0;
    for (int a : freeA) natural &= C->label[k++] == A->label[a];
    for (int b : freeB) natural &= C->label[k++] == B->label[b];
  }
  // permuted operand blocks: A block -> [freeA][con], B block -> [freeB][con (A's order)]
  auto dims_of = [](const QTensor& q, int blk, const std::vector<int>& axes) {
    int64_t n = 1;
    for (int k : axes) n *= q.sp[k].dim[q.blocks[blk][k]];
    return n;
  };
  std::vector<int64_t> aoff(qa.blocks.size()), boff(qb.blocks.size());
  int64_t ap_elems = 0, bp_elems = 0;
  for (size_t a = 0; a < qa.blocks.size(); ++a) {
    aoff[a] = ap_elems;
    ap_elems += dims_of(qa, (int)a, freeA) * dims_of(qa, (int)a, conA);
  }
  for (size_t b = 0; b < qb.blocks.size(); ++b) {
    boff[b] = bp_elems;
    bp_elems += dims_of(qb, (int)b, freeB) * dims_of(qb, (int)b, conB);
  }
  // grouped problems: one per reached C block
  std::vector<GProb> probs;
  std::vector<GSeg> segs;
  std::vector<GTile> tiles;
  std::vector<int64_t> toff(qc.blocks.size(), -1);  // natural-order result of each C block
  int64_t t_elems = 0;
  const int tile_cfg = 1;  // 128 x 128 register-staged tiles (any alignment)
  const int TR = grouped_tile_rows(tile_cfg), TC = grouped_tile_cols(P, tile_cfg);
  for (auto& kv : by_c) {
    const int cb = kv.first;
    const int a0 = kv.second[0].a, b0 = kv.second[0].b;
    const int64_t M = dims_of(qa, a0, freeA), N = dims_of(qb, b0, freeB);
    GProb pr{};
    pr.M = (int32_t)M;
    pr.N = (int32_t)N;
    pr.ldc = (int32_t)N;
    if (natural) {
      pr.c_off = qc.off[cb];
    } else {
      toff[cb] = t_elems;
      pr.c_off = t_elems;
      t_elems += M * N;
    }
    pr.seg0 = (int32_t)segs.size();
    pr.nseg = (int32_t)kv.second.size();
    pr.tiles_n = (int32_t)((N + TC - 1) / TC);
    pr.row0 = -1;
    for (const Pair& q : kv.second) {
      const int64_t K = dims_of(qa, q.a, conA);
      GSeg sg{};
      sg.a_off = aoff[q.a];
      sg.b_off = boff[q.b];
      sg.lda = (int32_t)K;
      sg.ldb = (int32_t)K;
      sg.K = (int32_t)K;
      segs.push_back(sg);
    }
    const int pi = (int)probs.size();
    probs.push_back(pr);
    for (int tm = 0; tm < (M + TR - 1) / TR; ++tm)
      for (int tn = 0; tn < pr.tiles_n; ++tn) tiles.push_back(GTile{pi, tm, tn, 0});
  }
  // the block permutations (operand blocks into K-contiguous matrices, and
  // the result blocks into C's label order), each set in one launch
  std::set<int> usedA, usedB;
  for (auto& kv : by_c)
    for (const Pair& q : kv.second) usedA.insert(q.a), usedB.insert(q.b);
  std::vector<PermItem> items;
  std::vector<PermChunk> chunks;
  auto add_item = [&](int64_t src, int64_t dst, const std::vector<int64_t>& od,
                      const std::vector<int64_t>& is) {
    PermItem it{};
    it.src = src;
    it.dst = dst;
    it.rank = (int32_t)od.size();
    it.n = 1;
    for (size_t k = 0; k < od.size(); ++k) it.dims[k] = od[k], it.istr[k] = is[k], it.n *= od[k];
    for (int64_t f = 0; f < it.n; f += PERM_CHUNK) chunks.push_back(PermChunk{(int32_t)items.size(), 0, f});
    items.push_back(it);
  };
  auto block_items = [&](const itn_tensor* t, const QTensor& q, const std::vector<int>& fr,
                         const std::vector<int>& cn, const std::vector<int64_t>& doff,
                         const std::set<int>& used) {
    for (size_t b = 0; b < q.blocks.size(); ++b) {
      if (!used.count((int)b)) continue;
      std::vector<int64_t> dims(t->rank), st(t->rank);
      for (int k = 0; k < t->rank; ++k) dims[k] = q.sp[k].dim[q.blocks[b][k]];
      int64_t acc = 1;
      for (int k = t->rank - 1; k >= 0; --k) {
        st[k] = acc;
        acc *= dims[k];
      }
      std::vector<int64_t> od, is;
      for (int k : fr) od.push_back(dims[k]), is.push_back(st[k]);
      for (int k : cn) od.push_back(dims[k]), is.push_back(st[k]);
      if (od.empty()) od.push_back(1), is.push_back(0);
      add_item(q.off[b], doff[b], od, is);
    }
  };
  block_items(A, qa, freeA, conA, aoff, usedA);
  const int64_t nchA = (int64_t)chunks.size();
  block_items(B, qb, freeB, conB, boff, usedB);
  const int64_t nchB = (int64_t)chunks.size() - nchA;
  if (!natural) {
    // T[cb] is [freeA..., freeB...]; each gathered into C's label order
    for (auto& kv : by_c) {
      const int cb = kv.first;
      const int a0 = kv.second[0].a, b0 = kv.second[0].b;
      std::vector<int64_t> tdims;
      for (int k : freeA) tdims.push_back(qa.sp[k].dim[qa.blocks[a0][k]]);
      for (int k : freeB) tdims.push_back(qb.sp[k].dim[qb.blocks[b0][k]]);
      std::vector<int64_t> tstr(tdims.size());
      int64_t acc = 1;
      for (int k = (int)tdims.size() - 1; k >= 0; --k) tstr[k] = acc, acc *= tdims[k];
      std::vector<int64_t> od(C->rank), is(C->rank);
      for (int k = 0; k < C->rank; ++k) {
        int pos = -1;
        for (size_t x = 0; x < freeA.size(); ++x)
          if (A->label[freeA[x]] == C->label[k]) pos = (int)x;
        for (size_t x = 0; x < freeB.size(); ++x)
          if (B->label[freeB[x]] == C->label[k]) pos = (int)(freeA.size() + x);
        od[k] = qc.sp[k].dim[qc.blocks[cb][k]];
        is[k] = tstr[pos];
      }
      if (od.empty()) od.push_back(1), is.push_back(0);
      add_item(toff[cb], qc.off[cb], od, is);
    }
  }
  const int64_t nchC = (int64_t)chunks.size() - nchA - nchB;
  // workspace: Ap, Bp, T, tables
  const size_t bAp = round256((size_t)std::max<int64_t>(ap_elems, 1) * es);
  const size_t bBp = round256((size_t)std::max<int64_t>(bp_elems, 1) * es);
  const size_t bT = round256((size_t)std::max<int64_t>(t_elems, 1) * dtype_size(acc_dt));
  const size_t bP = round256(std::max<size_t>(probs.size(), 1) * sizeof(GProb));
  const size_t bS = round256(std::max<size_t>(segs.size(), 1) * sizeof(GSeg));
  const size_t bTl = round256(std::max<size_t>(tiles.size(), 1) * sizeof(GTile));
  const size_t bB = round256(sizeof(GBases));
  const size_t bIt = round256(std::max<size_t>(items.size(), 1) * sizeof(PermItem));
  const size_t bCh = round256(std::max<size_t>(chunks.size(), 1) * sizeof(PermChunk));
  ITN_TRY(ensure_workspace(h, bAp + bBp + bT + bP + bS + bTl + bB + bIt + bCh + 256));
  Carver cv(h->ws.ptr);
  void* Ap = cv.take(bAp);
  void* Bp = cv.take(bBp);
  void* T = cv.take(bT);
  GProb* dprob = static_cast<GProb*>(cv.take(bP));
  GSeg* dseg = static_cast<GSeg*>(cv.take(bS));
  GTile* dtile = static_cast<GTile*>(cv.take(bTl));
  GBases* dbase = static_cast<GBases*>(cv.take(bB));
  PermItem* ditem = static_cast<PermItem*>(cv.take(bIt));
  PermChunk* dchunk = static_cast<PermChunk*>(cv.take(bCh));
  Prof pf(h, "qn_contract", s);
  // zero every C block no pair reaches (and all of C when there are none)
  for (size_t cb = 0; cb < qc.blocks.size(); ++cb)
    if (!by_c.count((int)cb)) {
      int64_t sz = 1;
      for (int k = 0; k < C->rank; ++k) sz *= qc.sp[k].dim[qc.blocks[cb][k]];
      ITN_HIP(h, fill(static_cast<char*>(C->data) + qc.off[cb] * dtype_size(C->dtype), C->dtype, 0.0, sz, s));
    }
  if (probs.empty()) return ITN_OK;
  // operand blocks permuted (and converted) into K-contiguous matrices
  ITN_HIP(h, hipMemcpyAsync(ditem, items.data(), items.size() * sizeof(PermItem), hipMemcpyHostToDevice, s));
  ITN_HIP(h, hipMemcpyAsync(dchunk, chunks.data(), chunks.size() * sizeof(PermChunk),
                            hipMemcpyHostToDevice, s));
  ITN_HIP(h, permute_batch(A->dtype, A->data, pt, Ap, ditem, dchunk, nchA, s));
  ITN_HIP(h, permute_batch(B->dtype, B->data, pt, Bp, ditem, dchunk + nchA, nchB, s));
  GBases gb{};
  gb.A = Ap;
  gb.B = Bp;
  gb.C = natural ? C->data : T;
  gb.zero = nullptr;
  gb.rows = nullptr;
  ITN_HIP(h, hipMemcpyAsync(dprob, probs.data(), probs.size() * sizeof(GProb), hipMemcpyHostToDevice, s));
  ITN_HIP(h, hipMemcpyAsync(dseg, segs.data(), segs.size() * sizeof(GSeg), hipMemcpyHostToDevice, s));
  ITN_HIP(h, hipMemcpyAsync(dtile, tiles.data(), tiles.size() * sizeof(GTile), hipMemcpyHostToDevice, s));
  ITN_HIP(h, hipMemcpyAsync(dbase, &gb, sizeof(GBases), hipMemcpyHostToDevice, s));
  ITN_HIP(h, gemm_grouped(P, natural ? C->dtype : acc_dt, tile_cfg, dbase, dprob, dseg, dtile,
                          (int64_t)tiles.size(), 0, 0, 0, 1, 0, s));
  if (!natural) ITN_HIP(h, permute_batch(acc_dt, T, C->dtype, C->data, ditem, dchunk + nchA + nchB, nchC, s));
  return ITN_OK;
}

}  // namespace itn
