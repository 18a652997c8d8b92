// Block-sparse (quantum-number) H_eff*psi: the integer host planner and the
// grouped, graph-captured execution.
//
// Sec. 8 fixes the rules the planner applies: an index is a list of QN
// sectors with an arrow; a block is stored iff Out QNs minus In QNs equal
// the tensor's flux; contracted indices need opposite arrows.  Sec. 9.4
// describes block-sparse contraction as dense contractions of block pairs,
// with several pairs possibly landing on one output block, and the option
// of combining blocks before contracting.  Here:
//   stage 1  one GEMM per (a-sector, m0-sector) group: the L block times all
//            psi blocks with that a-sector, concatenated along N (combine-
//            then-contract);
//   W-stage  per (a'-sector, b-sector) pair, a sparse map from the X blocks
//            to the Z blocks stage 4 needs;
//   stage 4  one problem per output block, its K the concatenation of the
//            (m2, b) segments of every contributing (Z block, R block) pair,
//            summed in ascending m2-sector order by the workgroup that owns
//            the output tile (no atomics: run-to-run deterministic).
#include <algorithm>
#include <array>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <tuple>
#include <unordered_map>
#include <mutex>
#include <sstream>

#include "handle.h"
#include "qn_common.h"

using namespace itn;
using namespace itn::qn;

namespace {

// Read a QN tensor: spaces, expected arrows, block list (validated).
itn_status read_qtensor(itn_handle* h, const itn_tensor* t, int rank, const int* arrows,
                        QTensor& out, const char* what, bool need_blocks) {
  if (!t) return fail(h, ITN_E_ARG, "%s is NULL", what);
  if (t->rank != rank) return fail(h, ITN_E_SHAPE, "%s must have rank %d", what, rank);
  if (!t->space) return fail(h, ITN_E_ARG, "%s needs QN index spaces", what);
  out.rank = rank;
  out.sp.resize(rank);
  for (int i = 0; i < rank; ++i) {
    ITN_TRY(read_space(h, t->space[i], out.sp[i], what));
    if (out.sp[i].arrow != arrows[i])
      return fail(h, ITN_E_ARROW, "%s index %d has arrow %d, expected %d", what, i, out.sp[i].arrow,
                  arrows[i]);
    if (out.sp[i].nq != out.sp[0].nq) return fail(h, ITN_E_SHAPE, "%s: mixed QN lengths", what);
    if (out.sp[i].mod != out.sp[0].mod) return fail(h, ITN_E_SHAPE, "%s: mixed QN addition rules", what);
  }
  if (!need_blocks) return ITN_OK;
  if (t->nblocks < 0 || (t->nblocks > 0 && (!t->block_sec || !t->block_off)))
    return fail(h, ITN_E_ARG, "%s: block list missing", what);
  const int nq = out.sp[0].nq;
  std::vector<int32_t> flux(nq, 0);
  if (t->flux) flux.assign(t->flux, t->flux + nq);
  for (int c = 0; c < nq; ++c)
    if (qn_red(flux[c], out.sp[0].mod[c]) != 0) return fail(h, ITN_E_FLUX, "%s must have zero flux", what);
  flux.assign(nq, 0);
  int64_t expect = 0;
  for (int64_t b = 0; b < t->nblocks; ++b) {
    std::vector<int32_t> blk(t->block_sec + b * rank, t->block_sec + (b + 1) * rank);
    int64_t sz = 1;
    for (int i = 0; i < rank; ++i) {
      if (blk[i] < 0 || blk[i] >= out.sp[i].nsec)
        return fail(h, ITN_E_ARG, "%s block %lld: sector out of range", what, (long long)b);
      sz *= out.sp[i].dim[blk[i]];
    }
    if (b > 0 && !(out.blocks.back() < blk))
      return fail(h, ITN_E_ARG, "%s blocks must be sorted and unique", what);
    if (block_flux(out, blk) != flux)
      return fail(h, ITN_E_FLUX, "%s block %lld violates the flux rule", what, (long long)b);
    if (t->block_off[b] != expect)
      return fail(h, ITN_E_SHAPE, "%s block offsets must be the exclusive prefix sum of block sizes",
                  what);
    expect += sz;
    out.index[blk] = (int)out.blocks.size();
    out.blocks.push_back(blk);
    out.off.push_back(t->block_off[b]);
  }
  out.elems = expect;
  return ITN_OK;
}

// Number of flux-allowed blocks (zero flux) of t: the charge sums of the
// first half of the indices tallied, then matched against the second half's.
int64_t count_allowed(const QTensor& t) {
  const int nq = t.sp[0].nq, h = t.rank / 2;
  const std::vector<int32_t>& mod = t.sp[0].mod;
  auto sums = [&](int i0, int i1, const std::function<void(const std::vector<int64_t>&)>& f) {
    std::vector<int64_t> acc(nq, 0);
    std::function<void(int)> rec = [&](int i) {
      if (i == i1) {
        f(acc);
        return;
      }
      for (int k = 0; k < t.sp[i].nsec; ++k) {
        for (int c = 0; c < nq; ++c) acc[c] += t.sp[i].arrow * (int64_t)t.sp[i].q(k)[c];
        rec(i + 1);
        for (int c = 0; c < nq; ++c) acc[c] -= t.sp[i].arrow * (int64_t)t.sp[i].q(k)[c];
      }
    };
    rec(i0);
  };
  std::map<std::vector<int32_t>, int64_t> left;
  sums(0, h, [&](const std::vector<int64_t>& a) {
    std::vector<int32_t> r(nq);
    for (int c = 0; c < nq; ++c) r[c] = qn_red(a[c], mod[c]);
    ++left[r];
  });
  int64_t n = 0;
  sums(h, t.rank, [&](const std::vector<int64_t>& a) {
    std::vector<int32_t> r(nq);
    for (int c = 0; c < nq; ++c) r[c] = qn_red(-a[c], mod[c]);
    auto it = left.find(r);
    if (it != left.end()) n += it->second;
  });
  return n;
}

bool distinct_qns(const QSpace& s) {
  for (int i = 0; i < s.nsec; ++i)
    for (int j = i + 1; j < s.nsec; ++j)
      if (std::equal(s.q(i), s.q(i) + s.nq, s.q(j))) return false;
  return true;
}

std::string sig_of(const QTensor& t) {
  std::ostringstream o;
  for (auto& s : t.sp) {
    o << "[" << (int)s.arrow;
    for (size_t k = 0; k < s.qn.size(); ++k) o << "," << s.qn[k];
    o << "%";
    for (auto m : s.mod) o << m << ",";
    o << ";";
    for (auto dd : s.dim) o << dd << ",";
    o << "]";
  }
  o << "B" << t.blocks.size() << ":";
  for (auto& b : t.blocks)
    for (auto k : b) o << k << ",";
  return o.str();
}

// process-wide autotune cache: plan signature -> (stage-1 mode, stage-4
// mode, W-stage kernel); lines "key m1 m4 w" in ITN_AUTOTUNE_CACHE if set
std::mutex g_tune_mu;
std::map<size_t, std::array<int, 3>> g_tune;
bool g_tune_loaded = false;

void tune_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("ITN_AUTOTUNE_CACHE");
  if (!path) return;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    size_t k;
    int a, b, c = 0;
    if (!(is >> k >> a >> b)) continue;
    is >> c;
    g_tune[k] = {a, b, c};
  }
}

void tune_store(size_t key, int a, int b, int c) {
  g_tune[key] = {a, b, c};
  const char* path = std::getenv("ITN_AUTOTUNE_CACHE");
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << key << " " << a << " " << b << " " << c << "\n";
}

}  // namespace

struct itn_plan {
  int prec = 0, pt = 0, xt = 0;
  int psi_dt = 0, out_dt = 0;
  int nv = 1;
  int64_t out_elems = 0;
  std::string sig;  // operand structure signature (L, R, psi)
  std::string sigL, sigR, sigP;  // the parts of sig
  size_t sig_hash = 0;
  // host tables
  std::vector<std::vector<int32_t>> out_blocks;
  std::vector<int64_t> out_off;
  std::vector<GProb> p1, p4;
  std::vector<GSeg> s1, s4;
  // Tile lists of a grouped stage.  all[c]: every problem with the
  // register-staged tile c (0: 64x64, 1: 128x128); big: the problems large
  // enough for the 8-wave 256-row direct tile; rest[c]: the others with tile
  // c; mid: problems with both extents >= 96 that are not big, on the
  // 4-wave 128x128 direct tile, rest_mid: the remaining ones (64x64);
  // midall: every problem with both extents >= 96 on the 128x128 direct
  // tile, rest_midall: the others (64x64); narrow: problems with M >= 96
  // and N < 96 on the 4-wave 256x64 direct tile, rest_nar: what neither
  // midall (= big + mid) nor narrow takes (64x64).  Launch modes: 0, 1 = all[mode]; 2, 3 = big then
  // rest[mode - 2]; 4 = big, mid, rest_mid; 5 = midall, rest_midall;
  // 6 = midall, narrow, rest_nar; 7 = big, mid, narrow, rest_nar.
  static constexpr int kModes = 8;
  struct Tiles {
    std::vector<GTile> all[2], big, rest[2], mid, rest_mid, midall, rest_midall, narrow, rest_nar;
    GTile *d_all[2] = {nullptr, nullptr}, *d_big = nullptr, *d_rest[2] = {nullptr, nullptr};
    GTile *d_mid = nullptr, *d_rest_mid = nullptr, *d_midall = nullptr, *d_rest_midall = nullptr;
    GTile *d_narrow = nullptr, *d_rest_nar = nullptr;
    size_t count(int mode) const {
      switch (mode) {
        case 0: case 1: return all[mode].size();
        case 2: case 3: return big.size() + rest[mode - 2].size();
        case 4: return big.size() + mid.size() + rest_mid.size();
        case 5: return midall.size() + rest_midall.size();
        case 6: return midall.size() + narrow.size() + rest_nar.size();
        default: return big.size() + mid.size() + narrow.size() + rest_nar.size();
      }
    }
    bool usable(int mode) const {
      if (mode == 2 || mode == 3) return !big.empty();
      if (mode == 4) return !big.empty() && !mid.empty();
      if (mode == 5) return !midall.empty();
      if (mode == 6) return !narrow.empty();
      if (mode == 7) return !big.empty() && !narrow.empty();
      return true;
    }
  } tl1, tl4;
  std::vector<QnTBlock> tb;
  std::vector<int32_t> tbi;  // block of every transpose tile
  int64_t tb_tiles = 0;
  std::vector<QnWPair> wp;
  std::vector<QnWEnt> we;
  // W-stage kernel candidates: work items (one wave each) of 64, 128 or 256
  // vectors; one item list each, the autotuner picks wsel.
  static constexpr int kWNum = 3;
  static constexpr int kWCand[kWNum] = {64, 128, 256};
  std::vector<QnWItem> wi[kWNum];
  int wsel = 0;
  std::vector<int64_t> rows4;  // stage-4 row table: output offset of every product row
  std::vector<QnCopy> cp;  // L / R repacks into padded, aligned blocks
  std::vector<int64_t> zoff, zsize;
  int64_t psiT_elems = 0, X_elems = 0, Z_elems = 0, Lp_elems = 0, Rp_elems = 0;
  int64_t max_db = 0;  // widest right bond sector (padded)
  int64_t X_real = 0, Z_real = 0;  // X and Z elements without the b padding
  int64_t pairs1 = 0;
  double flops_gemm = 0.0, flops_w = 0.0, flops_s1 = 0.0;
  // device state
  int device = -1;
  char* dtab = nullptr;  // all tables
  QnDevPtrs* dptrs = nullptr;
  GProb *dp1 = nullptr, *dp4 = nullptr;
  GSeg *ds1 = nullptr, *ds4 = nullptr;
  QnTBlock* dtb = nullptr;
  int32_t* dtbi = nullptr;
  QnWPair* dwp = nullptr;
  QnWEnt* dwe = nullptr;
  QnWItem* dwi[kWNum] = {nullptr, nullptr, nullptr};
  int64_t* drows4 = nullptr;
  QnCopy* dcp = nullptr;
  int64_t* dzoff = nullptr;
  int64_t* dzsize = nullptr;
  void* psiT = nullptr;
  void* X = nullptr;
  void* Z = nullptr;
  void* Lp = nullptr;  // padded copies of the used L / R blocks
  void* Rp = nullptr;
  void* zero = nullptr;  // zero page for K tails of direct-to-LDS tiles
  int cfg1 = 0, cfg4 = 0;
  bool tuned = false;
  bool direct = false;  // launch without graph capture (plans used for a few applies only)
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // applies with prepared environments (itn_qn_prepare_env): their own graph
  // without the L/R repack
  hipGraph_t graph_pe = nullptr;
  hipGraphExec_t exec_pe = nullptr;
  bool env_ready = false;
  bool out_set = false;
  const void* envL = nullptr;  // environments of the last prepare
  const void* envR = nullptr;
  ~itn_plan() {
    if (device >= 0) {
      (void)hipDeviceSynchronize();
      if (exec) (void)hipGraphExecDestroy(exec);
      if (graph) (void)hipGraphDestroy(graph);
      if (exec_pe) (void)hipGraphExecDestroy(exec_pe);
      if (graph_pe) (void)hipGraphDestroy(graph_pe);
      if (cap) (void)hipStreamDestroy(cap);
      if (dtab) (void)hipFree(dtab);  // tables and work buffers: one allocation
    }
  }
};

namespace {

// Row strides and block offsets of the plan-owned operand layouts are
// rounded up to 8 elements (16 bytes at bf16) and the padding is zero, so
// every K step of the grouped GEMMs is a whole, aligned 16-byte load.
inline int64_t pad8(int64_t x) { return (x + 7) & ~int64_t(7); }

// Split a block copy into items of at most 32 rows.
void add_copy(std::vector<QnCopy>& v, int64_t in_off, int64_t out_off, int rows, int cols, int ld,
              int src) {
  for (int r0 = 0; r0 < rows; r0 += 32) {
    QnCopy c{};
    c.in_off = in_off + (int64_t)r0 * cols;
    c.out_off = out_off + (int64_t)r0 * ld;
    c.rows = std::min(32, rows - r0);
    c.cols = cols;
    c.ld_out = ld;
    c.src = src;
    v.push_back(c);
  }
}

// Tile list (bm x bn tiles) over the problems `use` selects, each run of
// row panels on one XCD.  The persistent launch runs list position i on XCD
// i % 8 (workgroups go to the XCDs in turn; the grid and the list are
// multiples of 8), so the list interleaves eight queues: products are cut
// into runs of row panels of at most 1/32 of the total work, the runs are
// dealt to the XCDs largest first, each to the least loaded one, and a
// queue holds its runs' tiles row panel by row panel.  The tiles of a run
// share one L2, which serves its operand panels to every tile after the
// first instead of each XCD fetching them again (stage 1 of the cylinder
// bond read its operands about ten times over from beyond the L2 with the
// tiles spread over all XCDs).  Queues shorter than the longest are padded
// with empty tiles (prob = -1).
std::vector<GTile> make_tiles(const std::vector<GProb>& probs, const std::vector<GSeg>& segs, int bm,
                              int bn, const std::vector<char>& use) {
  struct Job {
    int64_t work;  // tiles x K
    int p;
  };
  std::vector<Job> jobs;
  for (size_t p = 0; p < probs.size(); ++p) {
    if (!use[p]) continue;
    int64_t k = 0;
    for (int s = 0; s < probs[p].nseg; ++s) k += segs[probs[p].seg0 + s].K;
    const int64_t t = (int64_t)((probs[p].M + bm - 1) / bm) * ((probs[p].N + bn - 1) / bn);
    jobs.push_back({t * k, (int)p});
  }
  constexpr int NX = 8;
  // products larger than 1/32 of the total are cut into runs of row panels
  // of at most that size (so that eight queues can balance), each run a job
  int64_t total = 0;
  for (const Job& j : jobs) total += j.work;
  const int64_t cap = std::max<int64_t>(1, total / (4 * NX));
  struct Run {
    int64_t work;
    int p, i0, i1;  // row panels [i0, i1)
  };
  std::vector<Run> runs;
  for (const Job& j : jobs) {
    const GProb& pr = probs[j.p];
    const int tm = (pr.M + bm - 1) / bm;
    const int64_t per_panel = j.work / tm;
    const int step = (int)std::max<int64_t>(1, cap / std::max<int64_t>(1, per_panel));
    for (int i0 = 0; i0 < tm; i0 += step) {
      const int i1 = std::min(tm, i0 + step);
      runs.push_back({per_panel * (i1 - i0), j.p, i0, i1});
    }
  }
  std::stable_sort(runs.begin(), runs.end(), [](const Run& a, const Run& b) { return a.work > b.work; });
  std::vector<GTile> q[NX];
  int64_t load[NX] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (const Run& r : runs) {
    int x = 0;
    for (int y = 1; y < NX; ++y)
      if (load[y] < load[x]) x = y;
    load[x] += r.work;
    const int tn = (probs[r.p].N + bn - 1) / bn;
    for (int i = r.i0; i < r.i1; ++i)
      for (int c = 0; c < tn; ++c) q[x].push_back(GTile{r.p, i, c, 0});
  }
  size_t len = 0;
  for (int x = 0; x < NX; ++x) len = std::max(len, q[x].size());
  std::vector<GTile> out;
  out.reserve(len * NX);
  const GTile none{-1, 0, 0, 0};
  for (size_t k = 0; k < len; ++k)
    for (int x = 0; x < NX; ++x) out.push_back(k < q[x].size() ? q[x][k] : none);
  return out;
}

// Problems that go to the direct-to-LDS tile: both extents at least 3/4 of
// a 256 tile, and every segment 16-byte aligned (true of the padded plan
// layouts; checked anyway).
template <typename TL>
void build_tiles(TL& tl, const std::vector<GProb>& probs, const std::vector<GSeg>& segs, int prec,
                 int dtype) {
  const int e16 = 16 / dtype_size(dtype);
  const size_t np = probs.size();
  std::vector<char> all(np, 1), big(np, 0), rest(np, 1), mid(np, 0), rest_mid(np, 1), midall(np, 0),
      rest_midall(np, 1), narrow(np, 0), rest_nar(np, 1);
  for (size_t p = 0; p < np; ++p) {
    const GProb& pr = probs[p];
    bool aligned = true;
    for (int s = 0; aligned && s < pr.nseg; ++s) {
      const GSeg& g = segs[pr.seg0 + s];
      aligned = g.a_off % e16 == 0 && g.b_off % e16 == 0 && g.lda % e16 == 0 && g.ldb % e16 == 0;
    }
    // both extents at least 3/4 of the tile
    const bool b = aligned && pr.M >= 192 && pr.N >= 192;
    const bool m = aligned && pr.M >= 96 && pr.N >= 96;
    big[p] = b;
    rest[p] = !b;
    mid[p] = m && !b;
    rest_mid[p] = !m;
    midall[p] = m;
    rest_midall[p] = !m;
    narrow[p] = aligned && pr.M >= 96 && pr.N < 96;
    rest_nar[p] = !m && !narrow[p];
  }
  for (int c = 0; c < 2; ++c) {
    const int t = grouped_tile_rows(c);
    tl.all[c] = make_tiles(probs, segs, t, t, all);
    tl.rest[c] = make_tiles(probs, segs, t, t, rest);
  }
  tl.big = make_tiles(probs, segs, grouped_tile_rows(2), grouped_tile_cols(prec, 2), big);
  tl.mid = make_tiles(probs, segs, 128, 128, mid);
  tl.rest_mid = make_tiles(probs, segs, 64, 64, rest_mid);
  tl.midall = make_tiles(probs, segs, 128, 128, midall);
  tl.rest_midall = make_tiles(probs, segs, 64, 64, rest_midall);
  tl.narrow = make_tiles(probs, segs, grouped_tile_rows(4), grouped_tile_cols(prec, 4), narrow);
  tl.rest_nar = make_tiles(probs, segs, 64, 64, rest_nar);
}

// Every access the plan's tables describe stays inside its buffer, and the
// W-stage vectors are 16-byte aligned: checked once per plan, on the host,
// before any table reaches the device.
bool layout_ok(const itn_plan& pl, int64_t psi_elems) {
  // transposes: output rows of ld_out >= rows rounded up to 8, offsets multiples of 8
  // elements (the kernel writes whole 16-byte vectors up to that rounding)
  if (pl.psiT_elems % 8 != 0) return false;
  for (const QnTBlock& t : pl.tb) {
    if (t.rows <= 0 || t.cols <= 0 || t.in_ld < t.cols || t.ld_out < pad8(t.rows)) return false;
    if (t.ld_out % 8 != 0 || t.out_off % 8 != 0) return false;
    if (t.in_off + (int64_t)(t.rows - 1) * t.in_ld + t.cols > psi_elems) return false;
    if (t.out_off + (int64_t)(t.cols - 1) * t.ld_out + pad8(t.rows) > pl.psiT_elems) return false;
  }
  for (const QnCopy& c : pl.cp) {
    const int64_t lim = c.src ? pl.Rp_elems : pl.Lp_elems;
    if (c.cols > c.ld_out || c.out_off + (int64_t)(c.rows - 1) * c.ld_out + c.cols > lim) return false;
  }
  auto seg_ok = [](const GProb& pr, const GSeg& g, int64_t a_lim, int64_t b_lim) {
    return g.K <= g.lda && g.K <= g.ldb && g.a_off + (int64_t)pr.M * g.lda <= a_lim &&
           g.b_off + (int64_t)pr.N * g.ldb <= b_lim;
  };
  for (const GProb& pr : pl.p1) {
    if (pr.row0 >= 0 || pr.c_off + (int64_t)pr.M * pr.ldc > pl.X_elems || pr.N > pr.ldc) return false;
    for (int k = 0; k < pr.nseg; ++k)
      if (!seg_ok(pr, pl.s1[pr.seg0 + k], pl.Lp_elems, pl.psiT_elems)) return false;
  }
  for (const GProb& pr : pl.p4) {
    if (pr.row0 < 0 || pr.row0 + (int64_t)pr.M > (int64_t)pl.rows4.size()) return false;
    for (int64_t r = 0; r < pr.M; ++r)
      if (pl.rows4[pr.row0 + r] < 0 || pl.rows4[pr.row0 + r] + pr.N > psi_elems) return false;
    for (int k = 0; k < pr.nseg; ++k)
      if (!seg_ok(pr, pl.s4[pr.seg0 + k], pl.Z_elems, pl.Rp_elems)) return false;
  }
  for (const QnWPair& wp : pl.wp) {
    if (wp.da <= 0 || wp.db <= 0 || wp.db % 8 || wp.ne <= 0) return false;
    for (int e = wp.e0; e < wp.e0 + wp.ne; ++e) {
      const QnWEnt& en = pl.we[e];
      if ((en.off | en.astride) % 8) return false;
      if (en.off < 0 || en.off + (int64_t)(wp.da - 1) * en.astride + wp.db > pl.X_elems + pl.max_db) return false;
      if (en.end) {
        if ((en.zoff | en.zastride) % 8) return false;
        if (en.zoff < 0 || en.zoff + (int64_t)(wp.da - 1) * en.zastride + wp.db > pl.Z_elems) return false;
      }
    }
    if (!pl.we[wp.e0 + wp.ne - 1].end) return false;
  }
  return pl.X_elems % 8 == 0 && pl.Z_elems % 8 == 0;
}

// The compute precision and the signature that includes it.
void set_prec(itn_plan& pl, int prec) {
  pl.prec = prec;
  pl.pt = prec == ITN_P_F64 ? D_F64 : (prec == ITN_P_F32 ? D_F32 : D_BF16);
  // X (stage 1's output) is the W-stage's operand: stored at the operand
  // precision (bf16 for bf16 applies: half the bytes of the HBM-bound
  // W-stage), accumulated in f32 by the W-stage.
  pl.xt = pl.pt;
  pl.sig = pl.sigL + "|" + pl.sigR + "|" + pl.sigP + "|" + std::to_string(pl.nv) + "|" +
           std::to_string(prec);
  pl.sig_hash = std::hash<std::string>()(pl.sig);
}

// The precision-dependent lists of a plan whose structure is built: the
// W-stage items (16-byte vectors of X's type), one list per kernel candidate,
// and the tile lists of both grouped stages; then the layout check.
itn_status finish_plan(itn_handle* h, itn_plan& pl) {
  const int64_t V = 16 / dtype_size(pl.xt);
  for (int c = 0; c < itn_plan::kWNum; ++c) {
    pl.wi[c].clear();
    const int64_t chunk = itn_plan::kWCand[c];
    for (size_t pid = 0; pid < pl.wp.size(); ++pid) {
      const int64_t nvec = (int64_t)pl.wp[pid].da * pl.wp[pid].db / V;
      for (int64_t v0 = 0; v0 < nvec; v0 += chunk)
        pl.wi[c].push_back(QnWItem{(int32_t)pid, (int32_t)v0});
    }
  }
  if (!layout_ok(pl, pl.out_elems)) return fail(h, ITN_E_SHAPE, "internal plan layout check failed");
  build_tiles(pl.tl1, pl.p1, pl.s1, pl.prec, pl.pt);
  build_tiles(pl.tl4, pl.p4, pl.s4, pl.prec, pl.pt);
  return ITN_OK;
}

itn_status build_plan(itn_handle* h, const itn_tensor* Lt, const itn_tensor* W1t,
                      const itn_tensor* W2t, const itn_tensor* Rt, const itn_tensor* Pt, int nv,
                      int prec, itn_plan& pl) {
  static const int aL[3] = {+1, -1, -1}, aR[3] = {-1, +1, +1}, aP[4] = {+1, +1, +1, -1},
                   aW[4] = {+1, -1, +1, -1};
  QTensor L, R, P, W1, W2;
  ITN_TRY(read_qtensor(h, Lt, 3, aL, L, "L", true));
  ITN_TRY(read_qtensor(h, Rt, 3, aR, R, "R", true));
  ITN_TRY(read_qtensor(h, Pt, 4, aP, P, "psi", true));
  ITN_TRY(read_qtensor(h, W1t, 4, aW, W1, "W1", false));
  ITN_TRY(read_qtensor(h, W2t, 4, aW, W2, "W2", false));
  const int nq = P.sp[0].nq;
  for (QTensor* t : {&L, &R, &W1, &W2})
    if (t->sp[0].nq != nq) return fail(h, ITN_E_SHAPE, "all operands need the same QN length");
  for (QTensor* t : {&L, &R, &W1, &W2})
    if (t->sp[0].mod != P.sp[0].mod) return fail(h, ITN_E_SHAPE, "all operands need the same QN rules");
  const std::vector<int32_t>& qmod = P.sp[0].mod;
  // contracted pairs: equal sectors (arrows already checked opposite)
  if (!L.sp[2].same_sectors(P.sp[0])) return fail(h, ITN_E_SHAPE, "L's a and psi's a differ");
  if (!L.sp[0].same_sectors(P.sp[0])) return fail(h, ITN_E_SHAPE, "L's a' and psi's a differ");
  if (!R.sp[2].same_sectors(P.sp[3])) return fail(h, ITN_E_SHAPE, "R's b and psi's b differ");
  if (!R.sp[0].same_sectors(P.sp[3])) return fail(h, ITN_E_SHAPE, "R's b' and psi's b differ");
  if (!L.sp[1].same_sectors(W1.sp[0])) return fail(h, ITN_E_SHAPE, "L's m and W1's m_in differ");
  if (!W1.sp[1].same_sectors(W2.sp[0])) return fail(h, ITN_E_SHAPE, "W1's m_out and W2's m_in differ");
  if (!W2.sp[1].same_sectors(R.sp[1])) return fail(h, ITN_E_SHAPE, "W2's m_out and R's m differ");
  if (!W1.sp[2].same_sectors(P.sp[1]) || !W1.sp[3].same_sectors(P.sp[1]))
    return fail(h, ITN_E_SHAPE, "W1's site indices and psi's s1 differ");
  if (!W2.sp[2].same_sectors(P.sp[2]) || !W2.sp[3].same_sectors(P.sp[2]))
    return fail(h, ITN_E_SHAPE, "W2's site indices and psi's s2 differ");
  if (!distinct_qns(P.sp[0]) || !distinct_qns(P.sp[3]))
    return fail(h, ITN_E_UNSUPPORTED, "bond indices must have distinct sector QNs");
  // psi must hold every allowed block (the output block set is psi's); its
  // stored blocks are unique and allowed, so counting the allowed ones suffices
  if (count_allowed(P) != (int64_t)P.blocks.size())
    return fail(h, ITN_E_SHAPE, "psi must store every flux-allowed block");
  const int w = (int)W1.sp[0].total, d1 = (int)P.sp[1].total, d2 = (int)P.sp[2].total;
  if (W2.sp[0].total != w) return fail(h, ITN_E_SHAPE, "W1 and W2 bond dimensions differ");
  if (!W1t->data || !W2t->data || W1t->dtype != ITN_F64 || W2t->dtype != ITN_F64)
    return fail(h, ITN_E_DTYPE, "W1, W2 must be host F64 dense arrays");
  const double* w1 = static_cast<const double*>(W1t->data);
  const double* w2 = static_cast<const double*>(W2t->data);
  // the MPO tensors must respect their own charges (each block's flux
  // computed once, then looked up per nonzero entry)
  auto sectors_of = [](const QSpace& s) {
    std::vector<int> r((size_t)s.total);
    for (int k = 0; k < s.nsec; ++k)
      for (int64_t g = s.off[k]; g < s.off[k] + s.dim[k]; ++g) r[(size_t)g] = k;
    return r;
  };
  for (int which = 0; which < 2; ++which) {
    const QTensor& Wt = which ? W2 : W1;
    const double* wd = which ? w2 : w1;
    const int d = which ? d2 : d1;
    const std::vector<int> k0 = sectors_of(Wt.sp[0]), k1 = sectors_of(Wt.sp[1]), k2 = sectors_of(Wt.sp[2]),
                           k3 = sectors_of(Wt.sp[3]);
    const int n1 = Wt.sp[1].nsec, n2 = Wt.sp[2].nsec, n3 = Wt.sp[3].nsec;
    std::vector<int8_t> ok((size_t)Wt.sp[0].nsec * n1 * n2 * n3, -1);  // -1: not yet computed
    for (int a = 0; a < w; ++a)
      for (int b = 0; b < w; ++b)
        for (int sp = 0; sp < d; ++sp)
          for (int s = 0; s < d; ++s) {
            if (wd[((a * w + b) * d + sp) * d + s] == 0.0) continue;
            int8_t& f = ok[(((size_t)k0[a] * n1 + k1[b]) * n2 + k2[sp]) * n3 + k3[s]];
            if (f < 0) {
              const auto fl = block_flux(Wt, {k0[a], k1[b], k2[sp], k3[s]});
              f = std::all_of(fl.begin(), fl.end(), [](int32_t v) { return v == 0; }) ? 1 : 0;
            }
            if (!f)
              return fail(h, ITN_E_FLUX, "W%d has a nonzero entry outside its allowed blocks", which + 1);
          }
  }
  const QSpace& SA = P.sp[0];
  const QSpace& S1 = P.sp[1];
  const QSpace& S2 = P.sp[2];
  const QSpace& SB = P.sp[3];
  const QSpace& SM = L.sp[1];   // m0 sectors
  const QSpace& SM2 = R.sp[1];  // m2 sectors
  pl.psi_dt = Pt->dtype;
  pl.nv = nv;
  pl.out_elems = P.elems;
  pl.out_blocks = P.blocks;
  pl.out_off = P.off;
  pl.sigL = sig_of(L);
  pl.sigR = sig_of(R);
  pl.sigP = sig_of(P);
  set_prec(pl, prec);

  // Every b-sector is padded to a multiple of 8 columns in psiT, X, Z and
  // the R copies (zero padding), so the W-stage moves aligned 16-byte
  // vectors; the padded K columns of the Z x R products multiply zeros.
  auto dbp = [&](int ib) -> int64_t { return pad8(SB.dim[ib]); };

  // ---- psiT layout: groups by a-sector; within one, the column blocks in
  // (b, s1, s2) sector order, so that the X inputs of one W-stage pair
  // (a'-sector, b-sector) are one contiguous run of every X row
  const int nA = SA.nsec;
  std::vector<int64_t> N_ia(nA, 0), N_real(nA, 0), psiT_off(nA, 0), colbase(P.blocks.size(), 0);
  std::vector<size_t> corder(P.blocks.size());
  for (size_t b = 0; b < corder.size(); ++b) corder[b] = b;
  std::stable_sort(corder.begin(), corder.end(), [&](size_t x, size_t y) {
    const auto &kx = P.blocks[x], &ky = P.blocks[y];
    return std::make_tuple(kx[0], kx[3], kx[1], kx[2]) < std::make_tuple(ky[0], ky[3], ky[1], ky[2]);
  });
  for (size_t b : corder) {
    const auto& k = P.blocks[b];
    const int64_t ss = (int64_t)S1.dim[k[1]] * S2.dim[k[2]];
    colbase[b] = N_ia[k[0]];
    N_ia[k[0]] += ss * dbp(k[3]);
    N_real[k[0]] += ss * SB.dim[k[3]];
  }
  std::vector<int64_t> ldT(nA);
  int64_t acc = 0;
  for (int ia = 0; ia < nA; ++ia) {
    ldT[ia] = pad8(SA.dim[ia]);
    psiT_off[ia] = acc;
    acc += pad8(N_ia[ia] * ldT[ia]);
  }
  pl.psiT_elems = acc;
  int64_t tiles = 0;
  auto add_tblock = [&](int64_t in_off, int64_t out_off, int rows, int64_t cols, int64_t in_ld,
                        int64_t ld_out) {
    QnTBlock t{};
    t.in_off = in_off;
    t.rows = rows;
    t.cols = (int32_t)cols;
    t.in_ld = (int32_t)in_ld;
    t.ld_out = (int32_t)ld_out;
    t.out_off = out_off;
    t.tiles_c = (t.cols + 63) / 64;
    t.tile0 = (int32_t)tiles;
    const int64_t nt = (int64_t)((t.rows + 63) / 64) * t.tiles_c;
    tiles += nt;
    pl.tbi.insert(pl.tbi.end(), (size_t)nt, (int32_t)pl.tb.size());
    pl.tb.push_back(t);
  };
  for (size_t b = 0; b < P.blocks.size(); ++b) {
    const auto& k = P.blocks[b];
    const int64_t ss = (int64_t)S1.dim[k[1]] * S2.dim[k[2]], db = SB.dim[k[3]];
    const int64_t base = psiT_off[k[0]] + colbase[b] * ldT[k[0]];
    if (db == dbp(k[3])) {
      add_tblock(P.off[b], base, SA.dim[k[0]], ss * db, ss * db, ldT[k[0]]);
    } else {  // one transpose per (s1, s2): the padded columns stay zero
      for (int64_t j = 0; j < ss; ++j)
        add_tblock(P.off[b] + j * db, base + j * dbp(k[3]) * ldT[k[0]], SA.dim[k[0]], db, ss * db,
                   ldT[k[0]]);
    }
  }
  pl.tb_tiles = tiles;

  // ---- stage 1: one product per a-sector over all its m0-sectors
  // X[(a', m0), (s1, s2, b)] = sum_a L[(a', m0), a] psiT[(s1, s2, b), a]: the
  // L blocks (a'(m0), m0, a) of one a-sector stack along the rows (their
  // padded copies are consecutive), so they share the psiT operand in one
  // product; X group (a, m0) is the row range of its L block.
  std::map<std::pair<int, int>, std::pair<int64_t, int>> xgroup;  // -> (X offset, a'-sector)
  int64_t xacc = 0;
  for (int ia = 0; ia < nA; ++ia) {
    if (N_ia[ia] == 0) continue;
    GProb pr{};
    pr.c_off = xacc;
    pr.N = (int32_t)N_ia[ia];
    pr.ldc = (int32_t)N_ia[ia];
    pr.seg0 = (int32_t)pl.s1.size();
    pr.nseg = 1;
    pr.row0 = -1;
    GSeg sg{};
    sg.a_off = pl.Lp_elems;
    sg.b_off = psiT_off[ia];
    sg.lda = (int32_t)ldT[ia];
    sg.ldb = (int32_t)ldT[ia];
    sg.K = (int32_t)ldT[ia];
    int64_t Mtot = 0;
    for (int im = 0; im < SM.nsec; ++im) {
      // L[a':Out, m:In, a:In], zero flux: q(a') = q(m) + q(a)
      const int iap = SA.find(qadd(SM.q(im), SA.q(ia), qmod, +1));
      if (iap < 0) continue;
      auto it = L.index.find({iap, im, ia});
      if (it == L.index.end()) continue;
      const int64_t M = (int64_t)SA.dim[iap] * SM.dim[im];
      add_copy(pl.cp, L.off[it->second], pl.Lp_elems, (int)M, SA.dim[ia], (int)ldT[ia], 0);
      pl.Lp_elems += M * ldT[ia];  // a multiple of 8: the next block follows directly
      xgroup[{ia, im}] = {xacc, iap};
      xacc += M * N_ia[ia];
      pl.X_real += M * N_real[ia];
      Mtot += M;
      pl.flops_gemm += 2.0 * M * N_real[ia] * SA.dim[ia];
      pl.flops_s1 += 2.0 * M * N_real[ia] * SA.dim[ia];
      for (size_t b = 0; b < P.blocks.size(); ++b) pl.pairs1 += P.blocks[b][0] == ia;
    }
    if (Mtot == 0) continue;
    pr.M = (int32_t)Mtot;
    pl.s1.push_back(sg);
    pl.p1.push_back(pr);
  }
  pl.X_elems = xacc;

  // ---- stage 4: one product per b'-sector over all output blocks with it
  // out[(a', s1', s2'), b'] = sum_{m2, b} Z[(a', s1', s2'), (m2, b)] R[b', (m2, b)]:
  // the output blocks of one b' share the segments (m2, b) of R, so their Z
  // blocks stack along the rows of one Z matrix per segment and the product
  // writes its rows to the blocks through a row table.
  // Z blocks: key (ia', is1', is2', im2, ib) and Z offset; sorted by key after stage 4
  std::vector<std::pair<std::array<int32_t, 5>, int64_t>> zblock;
  std::map<int, int64_t> rpad;                      // R block -> padded copy offset
  int64_t zacc = 0;
  std::map<int, std::vector<size_t>> by_bp;  // b'-sector -> output blocks (psi order)
  for (size_t ob = 0; ob < P.blocks.size(); ++ob) by_bp[P.blocks[ob][3]].push_back(ob);
  for (auto& kv : by_bp) {
    const int ibp = kv.first;
    const std::vector<size_t>& obs = kv.second;
    struct Seg {
      int im2, ib;
      int rb;  // R block
    };
    std::vector<Seg> segs;
    for (int im2 = 0; im2 < SM2.nsec; ++im2) {
      // R[b':In, m:Out, b:Out], zero flux: q(b) = q(b') - q(m)
      const int ib = SB.find(qadd(SB.q(ibp), SM2.q(im2), qmod, -1));
      if (ib < 0) continue;
      auto it = R.index.find({ibp, im2, ib});
      if (it == R.index.end()) continue;
      segs.push_back(Seg{im2, ib, it->second});
    }
    if (segs.empty()) {  // no R block: these output blocks are zero
      for (size_t ob : obs) {
        const auto& k = P.blocks[ob];
        pl.zoff.push_back(P.off[ob]);
        pl.zsize.push_back((int64_t)SA.dim[k[0]] * S1.dim[k[1]] * S2.dim[k[2]] * SB.dim[ibp]);
      }
      continue;
    }
    const int64_t N = SB.dim[ibp];
    GProb pr{};
    pr.c_off = 0;
    pr.N = (int32_t)N;
    pr.ldc = (int32_t)N;
    pr.seg0 = (int32_t)pl.s4.size();
    pr.nseg = (int32_t)segs.size();
    pr.row0 = (int32_t)pl.rows4.size();
    std::vector<int64_t> rowstart;
    int64_t Mtot = 0;
    for (size_t ob : obs) {
      const auto& k = P.blocks[ob];
      const int64_t M = (int64_t)SA.dim[k[0]] * S1.dim[k[1]] * S2.dim[k[2]];
      rowstart.push_back(Mtot);
      for (int64_t r = 0; r < M; ++r) pl.rows4.push_back(P.off[ob] + r * N);
      Mtot += M;
    }
    pr.M = (int32_t)Mtot;
    for (const Seg& sgm : segs) {
      const int64_t ldK = (int64_t)SM2.dim[sgm.im2] * dbp(sgm.ib);
      const int64_t base = zacc;
      zacc += Mtot * ldK;
      for (size_t i = 0; i < obs.size(); ++i) {
        const auto& k = P.blocks[obs[i]];
        zblock.push_back({{k[0], k[1], k[2], sgm.im2, sgm.ib}, base + rowstart[i] * ldK});
      }
      if (!rpad.count(sgm.rb)) {
        // R block [b'][m2][b] -> rows (b', m2) of dbp(b) columns
        rpad[sgm.rb] = pl.Rp_elems;
        add_copy(pl.cp, R.off[sgm.rb], pl.Rp_elems, (int)(N * SM2.dim[sgm.im2]), SB.dim[sgm.ib],
                 (int)dbp(sgm.ib), 1);
        pl.Rp_elems += N * ldK;
      }
      GSeg sg{};
      sg.a_off = base;
      sg.lda = (int32_t)ldK;
      sg.b_off = rpad[sgm.rb];
      sg.ldb = (int32_t)ldK;
      sg.K = (int32_t)ldK;
      pl.s4.push_back(sg);
      const int64_t K = (int64_t)SM2.dim[sgm.im2] * SB.dim[sgm.ib];
      pl.Z_real += Mtot * K;
      pl.flops_gemm += 2.0 * Mtot * N * K;  // algorithmic (unpadded) work
    }
    pl.p4.push_back(pr);
  }
  pl.Z_elems = zacc;

  // ---- W-stage: pairs (a'-sector, b-sector) over the Z blocks needed
  // W12[m0, m2, s1', s2', s1, s2] = sum_m1 W1[m0, m1, s1', s1] W2[m1, m2, s2', s2]
  const size_t nW12 = (size_t)w * w * d1 * d1 * d2 * d2;
  std::vector<double> W12(nW12, 0.0);
  auto w12 = [&](int m0, int m2, int s1p, int s2p, int s1, int s2) -> double& {
    return W12[((((((size_t)m0 * w + m2) * d1 + s1p) * d2 + s2p) * d1 + s1) * d2) + s2];
  };
  for (int m0 = 0; m0 < w; ++m0)
    for (int m1 = 0; m1 < w; ++m1)
      for (int s1p = 0; s1p < d1; ++s1p)
        for (int s1 = 0; s1 < d1; ++s1) {
          const double a = w1[((m0 * w + m1) * d1 + s1p) * d1 + s1];
          if (a == 0.0) continue;
          for (int m2 = 0; m2 < w; ++m2)
            for (int s2p = 0; s2p < d2; ++s2p)
              for (int s2 = 0; s2 < d2; ++s2) {
                const double b = w2[((m1 * w + m2) * d2 + s2p) * d2 + s2];
                if (b != 0.0) w12(m0, m2, s1p, s2p, s1, s2) += a * b;
              }
        }
  // The nonzeros of W12 for each output (m2, s1', s2'), in the order the
  // entries of a Z row are emitted: by input block (m0, s1, s2 sectors),
  // then m0, s1, s2 within it.
  struct W12nz {
    int m0, s1, s2, in;  // in: the input block's (m0, s1, s2) sector triple, flattened
    double c;
  };
  std::vector<std::vector<W12nz>> wcol((size_t)w * d1 * d2);
  {
    std::vector<int> km(w), k1(d1), k2(d2);
    for (int k = 0; k < SM.nsec; ++k)
      for (int64_t g = SM.off[k]; g < SM.off[k] + SM.dim[k]; ++g) km[(size_t)g] = k;
    for (int k = 0; k < S1.nsec; ++k)
      for (int64_t g = S1.off[k]; g < S1.off[k] + S1.dim[k]; ++g) k1[(size_t)g] = k;
    for (int k = 0; k < S2.nsec; ++k)
      for (int64_t g = S2.off[k]; g < S2.off[k] + S2.dim[k]; ++g) k2[(size_t)g] = k;
    for (int m0 = 0; m0 < w; ++m0)
      for (int m2 = 0; m2 < w; ++m2)
        for (int s1p = 0; s1p < d1; ++s1p)
          for (int s2p = 0; s2p < d2; ++s2p)
            for (int s1 = 0; s1 < d1; ++s1)
              for (int s2 = 0; s2 < d2; ++s2) {
                const double cf = w12(m0, m2, s1p, s2p, s1, s2);
                if (cf == 0.0) continue;
                const int in = (km[m0] * S1.nsec + k1[s1]) * S2.nsec + k2[s2];
                wcol[((size_t)m2 * d1 + s1p) * d2 + s2p].push_back(W12nz{m0, s1, s2, in, cf});
              }
    for (auto& col : wcol)
      std::stable_sort(col.begin(), col.end(), [](const W12nz& x, const W12nz& y) {
        if (x.in != y.in) return x.in < y.in;
        if (x.m0 != y.m0) return x.m0 < y.m0;
        if (x.s1 != y.s1) return x.s1 < y.s1;
        return x.s2 < y.s2;
      });
  }
  std::vector<int> in_of((size_t)SM.nsec * S1.nsec * S2.nsec, -1);  // input block per sector triple
  // lookups: psi's blocks per (a, b) sector pair as (s1, s2, block) in
  // ascending (s1, s2) order (psi's block list is sorted); the a-sector with
  // q(a) = q(a') - q(m0) per (a', m0) (-1: none); X group per (a, m0)
  struct PB {
    int i1, i2, b;
  };
  std::unordered_map<int64_t, std::vector<PB>> pab;
  for (size_t b = 0; b < P.blocks.size(); ++b) {
    const auto& k = P.blocks[b];
    pab[(int64_t)k[0] * SB.nsec + k[3]].push_back(PB{k[1], k[2], (int)b});
  }
  std::vector<std::pair<int64_t, int>> xg_of((size_t)SA.nsec * SM.nsec, {0, -1});  // (X offset, a'-sector)
  for (const auto& kv : xgroup) xg_of[(size_t)kv.first.first * SM.nsec + kv.first.second] = kv.second;
  std::vector<int> ia_of((size_t)SA.nsec * SM.nsec);
  for (int iap = 0; iap < SA.nsec; ++iap)
    for (int im0 = 0; im0 < SM.nsec; ++im0)
      ia_of[(size_t)iap * SM.nsec + im0] = SA.find(qadd(SA.q(iap), SM.q(im0), qmod, -1));
  std::sort(zblock.begin(), zblock.end());  // keys are unique
  std::map<std::pair<int, int>, std::vector<size_t>> pairs;  // (a', b) -> Z blocks, in key order
  for (size_t z = 0; z < zblock.size(); ++z) pairs[{zblock[z].first[0], zblock[z].first[4]}].push_back(z);
  for (auto& kv : pairs) {
    const int iap = kv.first.first, ib = kv.first.second;
    QnWPair wpair{};
    wpair.e0 = (int32_t)pl.we.size();
    wpair.da = SA.dim[iap];
    const int64_t db = SB.dim[ib], dbw = dbp(ib);  // true and padded widths
    wpair.db = (int32_t)dbw;
    pl.max_db = std::max<int64_t>(pl.max_db, dbw);
    // the X inputs of this pair, in entry order (they do not depend on the Z row)
    struct InBlock {
      int im0, ia, i1, i2;
      int64_t xbase, colbase;
    };
    std::vector<InBlock> inputs;
    for (int im0 = 0; im0 < SM.nsec; ++im0) {
      // X group (ia, im0) with q(a) = q(a') - q(m0)
      const int ia = ia_of[(size_t)iap * SM.nsec + im0];
      if (ia < 0) continue;
      const auto& xg = xg_of[(size_t)ia * SM.nsec + im0];
      if (xg.second != iap) continue;
      const auto pl_ab = pab.find((int64_t)ia * SB.nsec + ib);
      if (pl_ab == pab.end()) continue;
      for (const PB& pb : pl_ab->second) inputs.push_back({im0, ia, pb.i1, pb.i2, xg.first, colbase[pb.b]});
    }
    for (size_t k = 0; k < inputs.size(); ++k)
      in_of[((size_t)inputs[k].im0 * S1.nsec + inputs[k].i1) * S2.nsec + inputs[k].i2] = (int)k;
    for (size_t zi : kv.second) {
      const auto& zk = zblock[zi].first;
      const int i1p = zk[1], i2p = zk[2], im2 = zk[3];
      const int64_t zoff = zblock[zi].second;
      const int64_t ds1p = S1.dim[i1p], ds2p = S2.dim[i2p], dm2 = SM2.dim[im2];
      const int64_t ldZ = dm2 * dbw;
      for (int s1l = 0; s1l < ds1p; ++s1l)
        for (int s2l = 0; s2l < ds2p; ++s2l)
          for (int m2l = 0; m2l < dm2; ++m2l) {
            const int64_t row_off = zoff + (s1l * ds2p + s2l) * ldZ + m2l * dbw;
            const int64_t row_astride = ds1p * ds2p * ldZ;
            const size_t row_e0 = pl.we.size();
            const int g_m2 = (int)SM2.off[im2] + m2l;
            const int g_s1p = (int)S1.off[i1p] + s1l, g_s2p = (int)S2.off[i2p] + s2l;
            for (const W12nz& z : wcol[((size_t)g_m2 * d1 + g_s1p) * d2 + g_s2p]) {
              const int k = in_of[(size_t)z.in];
              if (k < 0) continue;
              const InBlock& in = inputs[(size_t)k];
              const int64_t ds2 = S2.dim[in.i2];
              const int64_t m0l = z.m0 - SM.off[in.im0], s1l2 = z.s1 - S1.off[in.i1], s2l2 = z.s2 - S2.off[in.i2];
              QnWEnt e{};
              e.off = in.xbase + m0l * N_ia[in.ia] + in.colbase + (s1l2 * ds2 + s2l2) * dbw;
              e.astride = (int64_t)SM.dim[in.im0] * N_ia[in.ia];
              e.coef = z.c;
              pl.we.push_back(e);
            }
            pl.flops_w += 2.0 * (double)(pl.we.size() - row_e0) * wpair.da * db;
            if (pl.we.size() == row_e0) {
              // no W12 term reaches this row: a zero-weight read of X[b] writes the zeros
              // (X is allocated max_db elements beyond its last vector)
              QnWEnt e{};
              pl.we.push_back(e);
            }
            QnWEnt& last = pl.we.back();
            last.zoff = row_off;
            last.zastride = row_astride;
            last.end = 1;
          }
    }
    for (const InBlock& in : inputs) in_of[((size_t)in.im0 * S1.nsec + in.i1) * S2.nsec + in.i2] = -1;
    wpair.ne = (int32_t)(pl.we.size() - wpair.e0);
    pl.wp.push_back(wpair);
  }
  return finish_plan(h, pl);
}

template <typename T> T* carve(char*& p, size_t n) {
  T* r = reinterpret_cast<T*>(p);
  p += (n * sizeof(T) + 255) & ~size_t(255);
  return r;
}

itn_status upload(itn_handle* h, itn_plan& pl) {
  pl.device = h->device;
  size_t bytes = 0;
  auto add = [&](size_t n) { bytes += (n + 255) & ~size_t(255); };
  add(sizeof(QnDevPtrs));
  add(pl.p1.size() * sizeof(GProb));
  add(pl.p4.size() * sizeof(GProb));
  add(pl.s1.size() * sizeof(GSeg));
  add(pl.s4.size() * sizeof(GSeg));
  for (auto* tl : {&pl.tl1, &pl.tl4}) {
    for (int c = 0; c < 2; ++c) {
      add(tl->all[c].size() * sizeof(GTile));
      add(tl->rest[c].size() * sizeof(GTile));
    }
    for (auto* v : {&tl->big, &tl->mid, &tl->rest_mid, &tl->midall, &tl->rest_midall, &tl->narrow,
                    &tl->rest_nar})
      add(v->size() * sizeof(GTile));
  }
  add(pl.tb.size() * sizeof(QnTBlock));
  add(pl.tbi.size() * sizeof(int32_t));
  add(pl.wp.size() * sizeof(QnWPair));
  add(pl.we.size() * sizeof(QnWEnt));
  for (int c = 0; c < itn_plan::kWNum; ++c) add(pl.wi[c].size() * sizeof(QnWItem));
  add(pl.rows4.size() * sizeof(int64_t));
  add(pl.cp.size() * sizeof(QnCopy));
  add(pl.zoff.size() * 8);
  add(pl.zsize.size() * 8);
  // The work buffers follow the tables in the same allocation, each 256-byte
  // aligned; their padding must read as zero (never rewritten).
  const int es = dtype_size(pl.pt), xs = dtype_size(pl.xt);
  size_t wbytes = 0;
  auto wadd = [&](size_t n) {
    const size_t o = wbytes;
    wbytes += (std::max<size_t>(256, n) + 255) & ~size_t(255);
    return o;
  };
  const size_t o_psiT = wadd((size_t)pl.nv * pl.psiT_elems * es);
  // + max b-sector width: zero-weight W-stage entries read X[v * X_elems + b]
  const size_t o_X = wadd(((size_t)pl.nv * pl.X_elems + (size_t)pl.max_db) * xs);
  const size_t o_Z = wadd((size_t)pl.nv * pl.Z_elems * es);
  const size_t o_Lp = wadd((size_t)pl.Lp_elems * es), o_Rp = wadd((size_t)pl.Rp_elems * es);
  const size_t o_zero = wadd(256);
  ITN_HIP(h, hipMalloc(&pl.dtab, bytes + wbytes));
  // tables laid out in a host mirror, then one copy
  std::vector<char> host(bytes, 0);
  char* p = pl.dtab;
  pl.dptrs = carve<QnDevPtrs>(p, 1);
  auto put = [&](auto*& dst, const auto& vec) -> hipError_t {
    using E = typename std::remove_reference<decltype(vec)>::type::value_type;
    dst = carve<E>(p, vec.size());
    if (!vec.empty())
      std::memcpy(host.data() + (reinterpret_cast<char*>(dst) - pl.dtab), vec.data(), vec.size() * sizeof(E));
    return hipSuccess;
  };
  ITN_HIP(h, put(pl.dp1, pl.p1));
  ITN_HIP(h, put(pl.dp4, pl.p4));
  ITN_HIP(h, put(pl.ds1, pl.s1));
  ITN_HIP(h, put(pl.ds4, pl.s4));
  for (auto* tl : {&pl.tl1, &pl.tl4}) {
    for (int c = 0; c < 2; ++c) {
      ITN_HIP(h, put(tl->d_all[c], tl->all[c]));
      ITN_HIP(h, put(tl->d_rest[c], tl->rest[c]));
    }
    ITN_HIP(h, put(tl->d_big, tl->big));
    ITN_HIP(h, put(tl->d_mid, tl->mid));
    ITN_HIP(h, put(tl->d_rest_mid, tl->rest_mid));
    ITN_HIP(h, put(tl->d_midall, tl->midall));
    ITN_HIP(h, put(tl->d_rest_midall, tl->rest_midall));
    ITN_HIP(h, put(tl->d_narrow, tl->narrow));
    ITN_HIP(h, put(tl->d_rest_nar, tl->rest_nar));
  }
  ITN_HIP(h, put(pl.dtb, pl.tb));
  ITN_HIP(h, put(pl.dtbi, pl.tbi));
  ITN_HIP(h, put(pl.dwp, pl.wp));
  ITN_HIP(h, put(pl.dwe, pl.we));
  for (int c = 0; c < itn_plan::kWNum; ++c) ITN_HIP(h, put(pl.dwi[c], pl.wi[c]));
  ITN_HIP(h, put(pl.drows4, pl.rows4));
  ITN_HIP(h, put(pl.dcp, pl.cp));
  ITN_HIP(h, put(pl.dzoff, pl.zoff));
  ITN_HIP(h, put(pl.dzsize, pl.zsize));
  if (p - pl.dtab > (std::ptrdiff_t)bytes) return fail(h, ITN_E_WORKSPACE, "internal: plan tables overrun");
  ITN_HIP(h, hipMemcpy(pl.dtab, host.data(), bytes, hipMemcpyHostToDevice));
  char* w0 = pl.dtab + bytes;
  pl.psiT = w0 + o_psiT;
  pl.X = w0 + o_X;
  pl.Z = w0 + o_Z;
  pl.Lp = w0 + o_Lp;
  pl.Rp = w0 + o_Rp;
  pl.zero = w0 + o_zero;
  ITN_HIP(h, hipMemset(w0, 0, wbytes));
  ITN_HIP(h, hipDeviceSynchronize());
  return ITN_OK;
}

constexpr int MAX_WG = 1024;  // persistent grouped launches: at most 4 workgroups per CU

// X and Z go out with nontemporal stores when they are larger than half of
// the 256 MiB last-level cache: the next pass reads them from HBM anyway,
// and the stores then do not displace the operands that stay cached
// between applies (L, R, psi).  Smaller ones (the 86 MB chain bond) stay
// cached for the pass that reads them.
int32_t big_for_cache(double bytes) { return bytes > 128.0 * 1024 * 1024 ? 1 : 0; }
int32_t x_stream(const itn_plan& pl) {
  return big_for_cache((double)pl.nv * (double)pl.X_elems * dtype_size(pl.xt));
}
int32_t z_stream(const itn_plan& pl) {
  return big_for_cache((double)pl.nv * (double)pl.Z_elems * dtype_size(pl.pt));
}

// The launches of one apply (after the operand pointers are set).
// The W-stage with kernel candidate c.
hipError_t wstage_launch(itn_plan& pl, int c, hipStream_t s) {
  return qn_wstage(pl.xt, pl.X, pl.Z, pl.dwp, pl.dwe, pl.dwi[c], (int64_t)pl.wi[c].size(),
                   pl.X_elems, pl.Z_elems, pl.nv, itn_plan::kWCand[c], z_stream(pl), s);
}

// One grouped stage (0: stage 1, 1: stage 4) in launch mode `mode`.
hipError_t stage_launch(itn_plan& pl, int stage, int mode, hipStream_t s) {
  const bool s1 = stage == 0;
  const GBases* b = s1 ? &pl.dptrs->g1 : &pl.dptrs->g4;
  const GProb* P = s1 ? pl.dp1 : pl.dp4;
  const GSeg* S = s1 ? pl.ds1 : pl.ds4;
  const itn_plan::Tiles& T = s1 ? pl.tl1 : pl.tl4;
  const int cdt = s1 ? pl.xt : pl.out_dt;
  const int64_t a_bs = s1 ? 0 : pl.Z_elems, b_bs = s1 ? pl.psiT_elems : 0;
  const int64_t c_bs = s1 ? pl.X_elems : pl.out_elems;
  auto run = [&](int cfg, const GTile* t, size_t n) {
    return gemm_grouped(pl.prec, cdt, cfg, b, P, S, t, (int64_t)n, a_bs, b_bs, c_bs, pl.nv, MAX_WG, s);
  };
  hipError_t e = hipSuccess;
  switch (mode) {
    case 0: case 1: return run(mode, T.d_all[mode], T.all[mode].size());
    case 2: case 3:
      if ((e = run(2, T.d_big, T.big.size())) != hipSuccess) return e;
      return run(mode - 2, T.d_rest[mode - 2], T.rest[mode - 2].size());
    case 4:
      if ((e = run(2, T.d_big, T.big.size())) != hipSuccess) return e;
      if ((e = run(3, T.d_mid, T.mid.size())) != hipSuccess) return e;
      return run(0, T.d_rest_mid, T.rest_mid.size());
    case 5:
      if ((e = run(3, T.d_midall, T.midall.size())) != hipSuccess) return e;
      return run(0, T.d_rest_midall, T.rest_midall.size());
    case 6:
      if ((e = run(3, T.d_midall, T.midall.size())) != hipSuccess) return e;
      if ((e = run(4, T.d_narrow, T.narrow.size())) != hipSuccess) return e;
      return run(0, T.d_rest_nar, T.rest_nar.size());
    case 7:
      if ((e = run(2, T.d_big, T.big.size())) != hipSuccess) return e;
      if ((e = run(3, T.d_mid, T.mid.size())) != hipSuccess) return e;
      if ((e = run(4, T.d_narrow, T.narrow.size())) != hipSuccess) return e;
      return run(0, T.d_rest_nar, T.rest_nar.size());
  }
  return hipErrorInvalidValue;
}

itn_status launch_all(itn_handle* h, itn_plan& pl, hipStream_t s, int cfg1, int cfg4,
                      bool with_env = true) {
  QnPtrs* ptrs = &pl.dptrs->p;
  if (with_env) {  // L/R repack and psi transpose in one launch
    Prof pf(h, "qn_env_repack_psi_transpose", s);
    ITN_HIP(h, qn_prepare(pl.psi_dt, ptrs, pl.pt, pl.psiT, pl.dtb, pl.dtbi, pl.tb_tiles, pl.out_elems,
                          pl.psiT_elems, pl.nv, pl.Lp, pl.Rp, pl.dcp, (int64_t)pl.cp.size(), s));
  } else {
    Prof pf(h, "qn_psi_transpose", s);
    ITN_HIP(h, qn_block_transpose(pl.psi_dt, ptrs, pl.pt, pl.psiT, pl.dtb, pl.dtbi, pl.tb_tiles,
                                  pl.out_elems, pl.psiT_elems, pl.nv, s));
  }
  {
    Prof pf(h, "qn_stage1_grouped", s);
    ITN_HIP(h, stage_launch(pl, 0, cfg1, s));
  }
  {
    Prof pf(h, "qn_wstage", s);
    ITN_HIP(h, wstage_launch(pl, pl.wsel, s));
  }
  if (!pl.zoff.empty()) {
    Prof pf(h, "qn_zero_blocks", s);
    ITN_HIP(h, qn_zero_blocks(pl.out_dt, ptrs, pl.dzoff, pl.dzsize, (int)pl.zoff.size(),
                              pl.out_elems, pl.nv, s));
  }
  {
    Prof pf(h, "qn_stage4_grouped", s);
    ITN_HIP(h, stage_launch(pl, 1, cfg4, s));
  }
  return ITN_OK;
}

// Pick the faster tile per grouped stage by timing both on the real operands.
itn_status autotune(itn_handle* h, itn_plan& pl, hipStream_t s) {
  // ITN_QN_WSTAGE=64|128|256 fixes the W-stage work item (vectors)
  int wforce = -1;
  if (const char* f = std::getenv("ITN_QN_WSTAGE")) {
    const int t = std::atoi(f);
    for (int c = 0; c < itn_plan::kWNum; ++c)
      if (itn_plan::kWCand[c] == t) wforce = c;
    if (wforce < 0) return fail(h, ITN_E_ARG, "ITN_QN_WSTAGE=%s is not an applicable W-stage kernel", f);
    pl.wsel = wforce;
  }
  // ITN_QN_TILE_MODE="m1,m4" fixes the launch modes (tests and experiments)
  if (const char* fm = std::getenv("ITN_QN_TILE_MODE")) {
    int a = -1, b = -1;
    if (std::sscanf(fm, "%d,%d", &a, &b) == 2 && a >= 0 && a < itn_plan::kModes && b >= 0 &&
        b < itn_plan::kModes) {
      pl.cfg1 = a;
      pl.cfg4 = b;
      if (wforce < 0) pl.wsel = 0;
      pl.tuned = true;
      return ITN_OK;
    }
    return fail(h, ITN_E_ARG, "ITN_QN_TILE_MODE must be \"m1,m4\" with modes 0..7");
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load();
    auto it = g_tune.find(pl.sig_hash);
    if (it != g_tune.end() && it->second[0] >= 0 && it->second[0] < itn_plan::kModes &&
        it->second[1] >= 0 && it->second[1] < itn_plan::kModes && it->second[2] >= 0 &&
        it->second[2] < itn_plan::kWNum) {
      pl.cfg1 = it->second[0];
      pl.cfg4 = it->second[1];
      if (wforce < 0) pl.wsel = it->second[2];
      pl.tuned = true;
      return ITN_OK;
    }
  }
  hipEvent_t e0, e1;
  ITN_HIP(h, hipEventCreate(&e0));
  ITN_HIP(h, hipEventCreate(&e1));
  float best1 = 1e30f, best4 = 1e30f;
  for (int c = 0; c < itn_plan::kModes; ++c) {
    for (int stage = 0; stage < 2; ++stage) {
      if (!(stage == 0 ? pl.tl1 : pl.tl4).usable(c)) continue;
      float tot = 0.f;
      for (int rep = 0; rep < 3; ++rep) {
        ITN_HIP(h, hipEventRecord(e0, s));
        ITN_HIP(h, stage_launch(pl, stage, c, s));
        ITN_HIP(h, hipEventRecord(e1, s));
        ITN_HIP(h, hipEventSynchronize(e1));
        float ms = 0.f;
        ITN_HIP(h, hipEventElapsedTime(&ms, e0, e1));
        if (rep > 0) tot += ms;
      }
      if (stage == 0 && tot < best1) best1 = tot, pl.cfg1 = c;
      if (stage == 1 && tot < best4) best4 = tot, pl.cfg4 = c;
    }
  }
  if (wforce < 0) {  // W-stage kernel candidates
    float bestw = 1e30f;
    for (int c = 0; c < itn_plan::kWNum; ++c) {
      float tot = 0.f;
      for (int rep = 0; rep < 3; ++rep) {
        ITN_HIP(h, hipEventRecord(e0, s));
        ITN_HIP(h, wstage_launch(pl, c, s));
        ITN_HIP(h, hipEventRecord(e1, s));
        ITN_HIP(h, hipEventSynchronize(e1));
        float ms = 0.f;
        ITN_HIP(h, hipEventElapsedTime(&ms, e0, e1));
        if (rep > 0) tot += ms;
      }
      if (tot < bestw) bestw = tot, pl.wsel = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  pl.tuned = true;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_store(pl.sig_hash, pl.cfg1, pl.cfg4, pl.wsel);
  return ITN_OK;
}

}  // namespace

extern "C" {

itn_status itn_qn_heff_plan(itn_handle* h, const itn_tensor* L, const itn_tensor* W1,
                            const itn_tensor* W2, const itn_tensor* R, const itn_tensor* psi,
                            int32_t nv, itn_prec prec, itn_plan** plan) {
  if (!h) return ITN_E_ARG;
  if (!plan) return fail(h, ITN_E_ARG, "plan is NULL");
  *plan = nullptr;
  if (nv < 1) return fail(h, ITN_E_ARG, "nv must be >= 1");
  if (prec != ITN_P_F64 && prec != ITN_P_F32 && prec != ITN_P_BF16)
    return fail(h, ITN_E_ARG, "unknown precision");
  if (psi && psi->dtype != ITN_F64 && psi->dtype != ITN_F32)
    return fail(h, ITN_E_DTYPE, "psi must be F64 or F32");
  auto* pl = new itn_plan();
  itn_status st = build_plan(h, L, W1, W2, R, psi, nv, prec, *pl);
  if (st != ITN_OK) {
    delete pl;
    return st;
  }
  *plan = pl;
  return ITN_OK;
}

itn_status itn_qn_allowed_blocks(itn_handle* h, const itn_tensor* t, int64_t* nblocks,
                                 int32_t* block_sec, int64_t* block_off, int64_t* total) {
  if (!h) return ITN_E_ARG;
  if (!t || !nblocks || !total) return fail(h, ITN_E_ARG, "null argument");
  if (t->rank < 1 || t->rank > 8 || !t->space) return fail(h, ITN_E_ARG, "need 1..8 QN indices");
  QTensor q;
  q.rank = t->rank;
  q.sp.resize(t->rank);
  for (int i = 0; i < t->rank; ++i) {
    ITN_TRY(read_space(h, t->space[i], q.sp[i], "t"));
    if (q.sp[i].nq != q.sp[0].nq) return fail(h, ITN_E_SHAPE, "mixed QN lengths");
    if (q.sp[i].mod != q.sp[0].mod) return fail(h, ITN_E_SHAPE, "mixed QN addition rules");
  }
  const int nq = q.sp[0].nq;
  std::vector<int32_t> flux(nq, 0);
  if (t->flux) flux.assign(t->flux, t->flux + nq);
  for (int c = 0; c < nq; ++c) flux[c] = qn_red(flux[c], q.sp[0].mod[c]);
  std::vector<std::vector<int32_t>> out;
  std::vector<int32_t> blk(q.rank, 0);
  std::function<void(int)> rec = [&](int i) {
    if (i == q.rank) {
      if (block_flux(q, blk) == flux) out.push_back(blk);
      return;
    }
    for (int k = 0; k < q.sp[i].nsec; ++k) {
      blk[i] = k;
      rec(i + 1);
    }
  };
  rec(0);
  int64_t acc = 0;
  std::vector<int64_t> offs;
  for (auto& b : out) {
    offs.push_back(acc);
    int64_t sz = 1;
    for (int i = 0; i < q.rank; ++i) sz *= q.sp[i].dim[b[i]];
    acc += sz;
  }
  if (block_sec) {
    if (!block_off) return fail(h, ITN_E_ARG, "block_off is NULL");
    if (*nblocks < (int64_t)out.size()) return fail(h, ITN_E_ARG, "capacity %lld < %zu blocks",
                                                    (long long)*nblocks, out.size());
    for (size_t b = 0; b < out.size(); ++b) {
      for (int i = 0; i < q.rank; ++i) block_sec[b * q.rank + i] = out[b][i];
      block_off[b] = offs[b];
    }
  }
  *nblocks = (int64_t)out.size();
  *total = acc;
  return ITN_OK;
}

itn_status itn_plan_destroy(itn_plan* plan) {
  delete plan;
  return ITN_OK;
}

}  // extern "C"

namespace itn {
// Fix a plan's launch modes (no autotuning) and launch it without graph
// capture: for plans that serve a handful of applies, as in a sweep.
itn_status qn_plan_at_prec(itn_handle* h, const itn_plan* src, int prec, itn_plan** out) {
  if (!h || !src || !out) return h ? fail(h, ITN_E_ARG, "null argument") : ITN_E_ARG;
  *out = nullptr;
  if (prec != ITN_P_F64 && prec != ITN_P_F32 && prec != ITN_P_BF16)
    return fail(h, ITN_E_ARG, "unknown precision");
  if (src->device >= 0 || src->dtab) return fail(h, ITN_E_ARG, "the source plan is already on a device");
  auto* pl = new itn_plan(*src);  // host tables only: no device state to share
  set_prec(*pl, prec);
  itn_status st = finish_plan(h, *pl);
  if (st != ITN_OK) {
    delete pl;
    return st;
  }
  *out = pl;
  return ITN_OK;
}

itn_status qn_plan_set_direct(itn_plan* pl, int mode_stage1, int mode_stage4) {
  if (!pl || mode_stage1 < 0 || mode_stage1 >= itn_plan::kModes || mode_stage4 < 0 ||
      mode_stage4 >= itn_plan::kModes)
    return ITN_E_ARG;
  if (!pl->tl1.usable(mode_stage1) || !pl->tl4.usable(mode_stage4)) return ITN_E_ARG;
  pl->cfg1 = mode_stage1;
  pl->cfg4 = mode_stage4;
  pl->wsel = 0;
  pl->tuned = true;
  pl->direct = true;
  return ITN_OK;
}
}  // namespace itn

extern "C" {

itn_status itn_qn_heff_diag(itn_handle* h, const itn_tensor* Lt, const itn_tensor* W1t, const itn_tensor* W2t,
                            const itn_tensor* Rt, itn_tensor* out, void* hip_stream) {
  if (!h) return ITN_E_ARG;
  static const int aL[3] = {+1, -1, -1}, aR[3] = {-1, +1, +1}, aP[4] = {+1, +1, +1, -1},
                   aW[4] = {+1, -1, +1, -1};
  QTensor L, R, P, W1, W2;
  ITN_TRY(read_qtensor(h, Lt, 3, aL, L, "L", true));
  ITN_TRY(read_qtensor(h, Rt, 3, aR, R, "R", true));
  ITN_TRY(read_qtensor(h, out, 4, aP, P, "out", true));
  ITN_TRY(read_qtensor(h, W1t, 4, aW, W1, "W1", false));
  ITN_TRY(read_qtensor(h, W2t, 4, aW, W2, "W2", false));
  if (!L.sp[0].same_sectors(P.sp[0]) || !L.sp[2].same_sectors(P.sp[0]))
    return fail(h, ITN_E_SHAPE, "L's a', a and out's a differ");
  if (!R.sp[0].same_sectors(P.sp[3]) || !R.sp[2].same_sectors(P.sp[3]))
    return fail(h, ITN_E_SHAPE, "R's b', b and out's b differ");
  if (!L.sp[1].same_sectors(W1.sp[0])) return fail(h, ITN_E_SHAPE, "L's m and W1's m_in differ");
  if (!W1.sp[1].same_sectors(W2.sp[0])) return fail(h, ITN_E_SHAPE, "W1's m_out and W2's m_in differ");
  if (!W2.sp[1].same_sectors(R.sp[1])) return fail(h, ITN_E_SHAPE, "W2's m_out and R's m differ");
  if (!W1.sp[2].same_sectors(P.sp[1]) || !W1.sp[3].same_sectors(P.sp[1]))
    return fail(h, ITN_E_SHAPE, "W1's site indices and out's s1 differ");
  if (!W2.sp[2].same_sectors(P.sp[2]) || !W2.sp[3].same_sectors(P.sp[2]))
    return fail(h, ITN_E_SHAPE, "W2's site indices and out's s2 differ");
  if (!W1t->data || !W2t->data || W1t->dtype != ITN_F64 || W2t->dtype != ITN_F64)
    return fail(h, ITN_E_DTYPE, "W1, W2 must be host F64 dense arrays");
  if (Lt->dtype != ITN_F64 || Rt->dtype != ITN_F64 || out->dtype != ITN_F64)
    return fail(h, ITN_E_DTYPE, "L, R and out must be F64");
  if (h->device < 0) return fail(h, ITN_E_NODEVICE, "host-only handle cannot launch work");
  if (P.elems == 0) return ITN_OK;
  if (!out->data || (!Lt->data && L.elems > 0) || (!Rt->data && R.elems > 0))
    return fail(h, ITN_E_ARG, "L, R and out need device data");
  HeffDiag dg;
  ITN_TRY(heff_diag_build(h, L, R, static_cast<const double*>(W1t->data), static_cast<const double*>(W2t->data),
                          (int)W1.sp[1].total, P, dg));
  ITN_TRY(ensure_workspace(h, dg.device_bytes()));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  ITN_HIP(h, heff_diag_launch(dg, static_cast<const double*>(Lt->data), static_cast<const double*>(Rt->data),
                              h->ws.ptr, static_cast<double*>(out->data), s));
  ITN_HIP(h, hipStreamSynchronize(s));  // the host tables go out of scope here
  return ITN_OK;
}

itn_status itn_plan_query(const itn_plan* pl, itn_plan_info* info) {
  if (!pl || !info) return ITN_E_ARG;
  info->out_nblocks = (int64_t)pl->out_blocks.size();
  info->out_elems = pl->out_elems;
  info->n_pairs_stage1 = pl->pairs1;
  info->n_groups_stage1 = (int64_t)pl->p1.size();
  info->n_pairs_stage4 = (int64_t)pl->s4.size();
  info->n_tiles = (int64_t)(pl->tl1.count(pl->cfg1) + pl->tl4.count(pl->cfg4));
  info->flops = pl->flops_gemm * pl->nv;
  info->x_elems = pl->X_real;
  info->z_elems = pl->Z_real;
  info->flops_wstage = pl->flops_w * pl->nv;
  info->flops_stage1 = pl->flops_s1 * pl->nv;
  info->mode_stage1 = pl->tuned ? pl->cfg1 : -1;
  info->mode_stage4 = pl->tuned ? pl->cfg4 : -1;
  info->wstage_tile = pl->tuned ? itn_plan::kWCand[pl->wsel] : -1;
  return ITN_OK;
}

itn_status itn_plan_out_blocks(const itn_plan* pl, int32_t* block_sec, int64_t* block_off) {
  if (!pl || !block_sec || !block_off) return ITN_E_ARG;
  for (size_t b = 0; b < pl->out_blocks.size(); ++b) {
    for (int i = 0; i < 4; ++i) block_sec[b * 4 + i] = pl->out_blocks[b][i];
    block_off[b] = pl->out_off[b];
  }
  return ITN_OK;
}

// Structure and dtype checks of environments against the plan.
static itn_status check_env(itn_handle* h, const itn_plan* pl, const itn_tensor* L, const itn_tensor* R) {
  static const int aL[3] = {+1, -1, -1}, aR[3] = {-1, +1, +1};
  QTensor Lq, Rq;
  ITN_TRY(read_qtensor(h, L, 3, aL, Lq, "L", true));
  ITN_TRY(read_qtensor(h, R, 3, aR, Rq, "R", true));
  if (sig_of(Lq) != pl->sigL || sig_of(Rq) != pl->sigR)
    return fail(h, ITN_E_SHAPE, "operands differ from the plan's structure");
  if (L->dtype != pl->pt || R->dtype != pl->pt)
    return fail(h, ITN_E_DTYPE, "L and R must be stored in the plan's compute type");
  return ITN_OK;
}

static itn_status ensure_device(itn_handle* h, itn_plan* pl) {
  if (h->device < 0) return fail(h, ITN_E_NODEVICE, "host-only handle cannot launch work");
  if (pl->device < 0) {
    ITN_TRY(upload(h, *pl));
  } else if (pl->device != h->device) {
    return fail(h, ITN_E_ARG, "plan was uploaded to another device");
  }
  return ITN_OK;
}

itn_status itn_qn_prepare_env(itn_handle* h, itn_plan* pl, const itn_tensor* L, const itn_tensor* R,
                              void* hip_stream) {
  if (!h) return ITN_E_ARG;
  if (!pl || !L || !R) return fail(h, ITN_E_ARG, "null argument");
  ITN_TRY(check_env(h, pl, L, R));
  ITN_TRY(ensure_device(h, pl));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  QnDevPtrs v{};
  v.p.L = L->data;
  v.p.R = R->data;
  v.g1 = GBases{pl->Lp, pl->psiT, pl->X, pl->zero, nullptr, x_stream(*pl), 0};
  v.g4 = GBases{pl->Z, pl->Rp, nullptr, pl->zero, pl->drows4, 0, 0};
  ITN_HIP(h, qn_set_ptrs(pl->dptrs, v, s));
  {
    Prof pf(h, "qn_env_repack", s);
    ITN_HIP(h, qn_block_copy(pl->pt, &pl->dptrs->p, pl->Lp, pl->Rp, pl->dcp, (int64_t)pl->cp.size(), s));
  }
  pl->envL = L->data;
  pl->envR = R->data;
  pl->env_ready = true;
  return ITN_OK;
}

itn_status itn_qn_heff_apply(itn_handle* h, itn_plan* pl, const itn_tensor* L, const itn_tensor* R,
                             const itn_tensor* psi, itn_tensor* out, void* hip_stream) {
  if (!h) return ITN_E_ARG;
  if (!pl || !psi || !out) return fail(h, ITN_E_ARG, "null argument");
  const bool prepared = !L && !R;
  if (!prepared && (!L || !R)) return fail(h, ITN_E_ARG, "pass both L and R, or neither (prepared)");
  if (prepared && !pl->env_ready)
    return fail(h, ITN_E_ARG, "no prepared environments: call itn_qn_prepare_env first");
  // operands must carry the structure the plan was built from
  {
    static const int aP[4] = {+1, +1, +1, -1};
    QTensor Pq, Oq;
    if (!prepared) ITN_TRY(check_env(h, pl, L, R));
    ITN_TRY(read_qtensor(h, psi, 4, aP, Pq, "psi", true));
    ITN_TRY(read_qtensor(h, out, 4, aP, Oq, "out", true));
    if (sig_of(Pq) != pl->sigP) return fail(h, ITN_E_SHAPE, "operands differ from the plan's structure");
    if (sig_of(Oq) != sig_of(Pq)) return fail(h, ITN_E_SHAPE, "out must have psi's structure");
  }
  if (psi->dtype != pl->psi_dt) return fail(h, ITN_E_DTYPE, "psi dtype differs from the plan's");
  if (out->dtype != ITN_F64 && out->dtype != ITN_F32)
    return fail(h, ITN_E_DTYPE, "out must be F64 or F32");
  ITN_TRY(ensure_device(h, pl));
  if (!pl->out_set) {
    pl->out_dt = out->dtype;
    pl->out_set = true;
  }
  if (out->dtype != pl->out_dt) return fail(h, ITN_E_DTYPE, "out dtype differs from the first apply");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  QnDevPtrs v{};
  v.p.L = prepared ? pl->envL : L->data;
  v.p.R = prepared ? pl->envR : R->data;
  v.p.psi = psi->data;
  v.p.out = out->data;
  v.g1 = GBases{pl->Lp, pl->psiT, pl->X, pl->zero, nullptr, x_stream(*pl), 0};
  v.g4 = GBases{pl->Z, pl->Rp, out->data, pl->zero, pl->drows4, 0, 0};
  {
    Prof pf(h, "qn_set_ptrs", s);
    ITN_HIP(h, qn_set_ptrs(pl->dptrs, v, s));
  }
  // an apply with environments repacks them: later prepared applies use these
  if (!prepared) {
    pl->envL = L->data;
    pl->envR = R->data;
    pl->env_ready = true;
  }
  if (!pl->tuned) ITN_TRY(autotune(h, *pl, s));
  if (h->prof_on || pl->direct) {  // per-kernel timing, or a short-lived plan: launch directly
    ITN_TRY(launch_all(h, *pl, s, pl->cfg1, pl->cfg4, !prepared));
    return ITN_OK;
  }
  hipGraph_t& graph = prepared ? pl->graph_pe : pl->graph;
  hipGraphExec_t& exec = prepared ? pl->exec_pe : pl->exec;
  if (!exec) {
    if (!pl->cap) ITN_HIP(h, hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking));
    ITN_HIP(h, hipStreamBeginCapture(pl->cap, hipStreamCaptureModeThreadLocal));
    const itn_status st = launch_all(h, *pl, pl->cap, pl->cfg1, pl->cfg4, !prepared);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(pl->cap, &g);
    if (st != ITN_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    ITN_HIP(h, e);
    graph = g;
    ITN_HIP(h, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  }
  ITN_HIP(h, hipGraphLaunch(exec, s));
  return ITN_OK;
}

}  // extern "C"
