// Plain and grouped NT GEMM kernels (MFMA, gfx950).
#include "gemm_core.h"
#include "kernels.h"

namespace itn {

template <int P, int BM, int BN, bool ALIGNED, typename TOut>
__global__ __launch_bounds__(GEMM_THREADS) void gemm_nt_kernel(GemmArgs g, int64_t tiles_m,
                                                                 int64_t tiles_n) {
  using Cfg = TileCfg<P, BM, BN>;
  using T = typename Cfg::T;
  extern __shared__ __align__(16) char lds[];
  int64_t tm, tn;
  tile_coords(blockIdx.x, tiles_m * tiles_n, tiles_m, tiles_n, tm, tn);
  const int64_t b = blockIdx.y;
  const T* A = static_cast<const T*>(g.A) + b * g.sA;
  const T* B = static_cast<const T*>(g.B) + b * g.sB;
  TOut* Cp = static_cast<TOut*>(g.C) + b * g.sC;
  typename Cfg::AccV acc[BM / 32][BN / 32];
  zero_acc<P, BM, BN>(acc);
  gemm_accum<P, BM, BN, ALIGNED>(A, g.lda, g.M, B, g.ldb, g.N, g.K, tm * BM, tn * BN, acc, lds);
  store_tile<P, BM, BN, TOut>(acc, Cp, g.ldc, g.M, g.N, tm * BM, tn * BN, g.accumulate != 0);
}

template <int P, int BM, int BN, int WM, int WN, typename TOut, int MODE>
__global__ __launch_bounds__(64 * WM * WN) void gemm_nt_direct_kernel(GemmArgs g, int64_t tiles_m,
                                                                        int64_t tiles_n) {
  using Cfg = DirectCfg<P, BM, BN, WM, WN>;
  using T = typename Cfg::T;
  extern __shared__ __align__(16) char lds[];
  int64_t tm, tn;
  tile_coords(blockIdx.x, tiles_m * tiles_n, tiles_m, tiles_n, tm, tn);
  const int64_t b = blockIdx.y;
  const T* A = static_cast<const T*>(g.A) + b * g.sA;
  const T* B = static_cast<const T*>(g.B) + b * g.sB;
  TOut* Cp = static_cast<TOut*>(g.C) + b * g.sC;
  typename Cfg::AccV acc[Cfg::FM][Cfg::FN];
#pragma unroll
  for (int i = 0; i < Cfg::FM; ++i)
#pragma unroll
    for (int j = 0; j < Cfg::FN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[i][j][e] = 0;
  gemm_accum_direct<P, BM, BN, WM, WN>(A, g.lda, g.M, B, g.ldb, g.N, g.K, tm * BM, tn * BN, acc, lds);
  store_tile_direct<P, BM, BN, WM, WN, TOut, MODE>(acc, Cp, g.ldc, g.M, g.N, tm * BM, tn * BN);
}

// Persistent grouped GEMM: gridDim.x workgroups stride over the tile list
// (ordered by the planner, largest work first); base pointers are read from
// device memory so that a captured graph can be replayed with new operands.
template <int P, int BM, int BN, typename TOut>
__global__ __launch_bounds__(GEMM_THREADS) void gemm_grouped_kernel(
    const GBases* __restrict__ bases, const GProb* __restrict__ probs, const GSeg* __restrict__ segs,
    const GTile* __restrict__ tiles, int64_t ntiles, int64_t a_bs, int64_t b_bs, int64_t c_bs) {
  using Cfg = TileCfg<P, BM, BN>;
  using T = typename Cfg::T;
  constexpr int E16 = Cfg::E16;
  extern __shared__ __align__(16) char lds[];
  const T* Abase = static_cast<const T*>(bases->A);
  const T* Bbase = static_cast<const T*>(bases->B);
  TOut* Cbase = static_cast<TOut*>(bases->C);
  const int64_t batch = blockIdx.y;
  for (int64_t ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
    const GTile t = tiles[ti];
    if (t.prob < 0) continue;  // padding that keeps every list position on its XCD
    const GProb pr = probs[t.prob];
    typename Cfg::AccV acc[BM / 32][BN / 32];
    zero_acc<P, BM, BN>(acc);
    for (int s = 0; s < pr.nseg; ++s) {
      const GSeg sg = segs[pr.seg0 + s];
      const T* A = Abase + sg.a_off + batch * a_bs;
      const T* B = Bbase + sg.b_off + batch * b_bs;
      // uniform over the workgroup (depends on the segment only)
      const bool al = ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) & 15) == 0 &&
                      sg.lda % E16 == 0 && sg.ldb % E16 == 0;
      if (al)
        gemm_accum<P, BM, BN, true>(A, sg.lda, pr.M, B, sg.ldb, pr.N, sg.K, (int64_t)t.tm * BM,
                                    (int64_t)t.tn * BN, acc, lds);
      else
        gemm_accum<P, BM, BN, false>(A, sg.lda, pr.M, B, sg.ldb, pr.N, sg.K, (int64_t)t.tm * BM,
                                     (int64_t)t.tn * BN, acc, lds);
    }
    const int64_t* rows = pr.row0 >= 0 ? bases->rows + pr.row0 : nullptr;
    store_tile<P, BM, BN, TOut>(acc, Cbase + (rows ? 0 : pr.c_off) + batch * c_bs, pr.ldc, pr.M,
                                pr.N, (int64_t)t.tm * BM, (int64_t)t.tn * BN, false, rows);
  }
}

// Persistent grouped GEMM on direct-to-LDS 8-wave tiles (large problems of a
// grouped launch).  K segments may end inside a K step (zero page).
template <int P, int BM, int BN, int WM, int WN, typename TOut>
__global__ __launch_bounds__(64 * WM * WN) void gemm_grouped_direct_kernel(
    const GBases* __restrict__ bases, const GProb* __restrict__ probs, const GSeg* __restrict__ segs,
    const GTile* __restrict__ tiles, int64_t ntiles, int64_t a_bs, int64_t b_bs, int64_t c_bs) {
  using Cfg = DirectCfg<P, BM, BN, WM, WN>;
  using T = typename Cfg::T;
  extern __shared__ __align__(16) char lds[];
  const T* Abase = static_cast<const T*>(bases->A);
  const T* Bbase = static_cast<const T*>(bases->B);
  const T* zero = static_cast<const T*>(bases->zero);
  TOut* Cbase = static_cast<TOut*>(bases->C);
  const int64_t batch = blockIdx.y;
  for (int64_t ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
    const GTile t = tiles[ti];
    if (t.prob < 0) continue;  // padding that keeps every list position on its XCD
    const GProb pr = probs[t.prob];
    typename Cfg::AccV acc[Cfg::FM][Cfg::FN];
#pragma unroll
    for (int i = 0; i < Cfg::FM; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::FN; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[i][j][e] = 0;
    for (int sgi = 0; sgi < pr.nseg; ++sgi) {
      const GSeg sg = segs[pr.seg0 + sgi];
      gemm_accum_direct<P, BM, BN, WM, WN, true>(Abase + sg.a_off + batch * a_bs, sg.lda, pr.M,
                                                 Bbase + sg.b_off + batch * b_bs, sg.ldb, pr.N, sg.K,
                                                 (int64_t)t.tm * BM, (int64_t)t.tn * BN, acc, lds, zero);
    }
    const int64_t* rows = pr.row0 >= 0 ? bases->rows + pr.row0 : nullptr;
    if constexpr (sizeof(TOut) == 2) {
      // whole-row 16-byte stores through LDS where C's rows are aligned (uniform per problem)
      if (!rows && ((pr.c_off | pr.ldc | pr.N | c_bs) & 7) == 0 &&
          (reinterpret_cast<uintptr_t>(Cbase) & 15) == 0) {
        if (bases->stream)
          store_tile_lds<P, BM, BN, WM, WN, TOut, true>(acc, Cbase + pr.c_off + batch * c_bs, pr.ldc,
                                                        pr.M, pr.N, (int64_t)t.tm * BM,
                                                        (int64_t)t.tn * BN, lds);
        else
          store_tile_lds<P, BM, BN, WM, WN, TOut, false>(acc, Cbase + pr.c_off + batch * c_bs, pr.ldc,
                                                         pr.M, pr.N, (int64_t)t.tm * BM,
                                                         (int64_t)t.tn * BN, lds);
        continue;
      }
    }
    store_tile_direct<P, BM, BN, WM, WN, TOut, 0>(acc, Cbase + (rows ? 0 : pr.c_off) + batch * c_bs,
                                                       pr.ldc, pr.M, pr.N, (int64_t)t.tm * BM,
                                                       (int64_t)t.tn * BN, rows);
  }
}

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// Tiles above 64 KiB of LDS need the per-kernel dynamic-LDS limit raised
// (gfx950 has 160 KiB per workgroup).
template <typename K> static hipError_t allow_lds(K kernel, int bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <int P, int BM, int BN, typename TOut>
static hipError_t launch_nt(const GemmArgs& g, hipStream_t s) {
  using Cfg = TileCfg<P, BM, BN>;
  const int64_t tiles_m = (g.M + BM - 1) / BM, tiles_n = (g.N + BN - 1) / BN;
  if (tiles_m == 0 || tiles_n == 0 || g.batch == 0) return hipSuccess;
  const int es = (int)sizeof(typename Cfg::T);
  const bool al = aligned16(g.A) && aligned16(g.B) && (g.lda * es) % 16 == 0 &&
                  (g.ldb * es) % 16 == 0 && (g.sA * es) % 16 == 0 && (g.sB * es) % 16 == 0;
  dim3 grid((unsigned)(tiles_m * tiles_n), (unsigned)g.batch);
  static const hipError_t attr =
      allow_lds(gemm_nt_kernel<P, BM, BN, true, TOut>, Cfg::LDS_BYTES) != hipSuccess
          ? hipErrorInvalidValue
          : allow_lds(gemm_nt_kernel<P, BM, BN, false, TOut>, Cfg::LDS_BYTES);
  if (attr != hipSuccess) return attr;
  if (al)
    hipLaunchKernelGGL((gemm_nt_kernel<P, BM, BN, true, TOut>), grid, dim3(GEMM_THREADS),
                       Cfg::LDS_BYTES, s, g, tiles_m, tiles_n);
  else
    hipLaunchKernelGGL((gemm_nt_kernel<P, BM, BN, false, TOut>), grid, dim3(GEMM_THREADS),
                       Cfg::LDS_BYTES, s, g, tiles_m, tiles_n);
  return hipGetLastError();
}

template <int P, int BM, int BN, int WM, int WN, typename TOut>
static hipError_t launch_nt_direct(const GemmArgs& g, hipStream_t s) {
  using Cfg = DirectCfg<P, BM, BN, WM, WN>;
  constexpr int LDS = Cfg::LDS_BYTES;
  const int64_t tiles_m = (g.M + BM - 1) / BM, tiles_n = (g.N + BN - 1) / BN;
  dim3 grid((unsigned)(tiles_m * tiles_n), (unsigned)g.batch);
  static const hipError_t attr =
      (allow_lds(gemm_nt_direct_kernel<P, BM, BN, WM, WN, TOut, 0>, LDS) != hipSuccess ||
       allow_lds(gemm_nt_direct_kernel<P, BM, BN, WM, WN, TOut, 1>, LDS) != hipSuccess)
          ? hipErrorInvalidValue
          : allow_lds(gemm_nt_direct_kernel<P, BM, BN, WM, WN, TOut, 2>, LDS);
  if (attr != hipSuccess) return attr;
  if (g.accumulate)
    hipLaunchKernelGGL((gemm_nt_direct_kernel<P, BM, BN, WM, WN, TOut, 1>), grid,
                       dim3(Cfg::THREADS), LDS, s, g, tiles_m, tiles_n);
  else if (g.stream)
    hipLaunchKernelGGL((gemm_nt_direct_kernel<P, BM, BN, WM, WN, TOut, 2>), grid,
                       dim3(Cfg::THREADS), LDS, s, g, tiles_m, tiles_n);
  else
    hipLaunchKernelGGL((gemm_nt_direct_kernel<P, BM, BN, WM, WN, TOut, 0>), grid,
                       dim3(Cfg::THREADS), LDS, s, g, tiles_m, tiles_n);
  return hipGetLastError();
}

// Direct-to-LDS tiles need 16-byte aligned rows and whole K steps.
template <int P> static bool direct_ok(const GemmArgs& g) {
  using T = typename PT<P>::T;
  const int es = (int)sizeof(T);
  const int64_t bk = ROW_BYTES / es;
  return aligned16(g.A) && aligned16(g.B) && (g.lda * es) % 16 == 0 && (g.ldb * es) % 16 == 0 &&
         (g.sA * es) % 16 == 0 && (g.sB * es) % 16 == 0 && g.K % bk == 0 && g.K > 0;
}

// Compute units of the current device (cached per device).
static int64_t device_cus() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cache[dev] == 0) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
      c = 256;
    cache[dev] = c;
  }
  return cache[dev];
}

template <int P, typename TOut>
static hipError_t dispatch_nt(const GemmArgs& g, hipStream_t s) {
  // Largest tile that still gives every CU at least one workgroup; small
  // problems use 64x64 tiles so that the launch spreads over the CUs.
  auto ntiles = [&](int bm, int bn) { return ((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn) * g.batch; };
  const int64_t cus = device_cus();
  // Direct-to-LDS tiles of 8 waves: 256 x 256 for 4-byte accumulators
  // (128 accumulator registers per lane); FP64 accumulators are twice as
  // wide, so FP64 uses 256 x 128.
  if constexpr (P == P_F64) {
    if (g.M >= 256 && g.N >= 128 && ntiles(256, 128) >= cus && direct_ok<P>(g))
      return launch_nt_direct<P, 256, 128, 2, 4, TOut>(g, s);
  } else {
    if (g.M >= 256 && g.N >= 256 && ntiles(256, 256) >= cus && direct_ok<P>(g)) {
      // Rounds of one tile per CU: a last round that fills a quarter of the
      // CUs costs a whole round.  192 x 256 tiles run at about 0.85 of the
      // 256 x 256 rate per flop (measured); take them when their rounds
      // cost less, e.g. M = 9 * 2048 (576 tiles of 256 x 256 = 2.25 rounds
      // against 768 of 192 x 256 = 3 full rounds).
      auto rounds = [&](int bm, int bn) { return (ntiles(bm, bn) + cus - 1) / cus; };
      const double c256 = (double)rounds(256, 256) * 256.0 * 256.0;
      const double c192 = (double)rounds(192, 256) * 192.0 * 256.0 / 0.85;
      if (c192 < c256) return launch_nt_direct<P, 192, 256, 2, 4, TOut>(g, s);
      return launch_nt_direct<P, 256, 256, 2, 4, TOut>(g, s);
    }
  }
  if (g.M >= 128 && g.N >= 128 && ntiles(128, 128) >= 256) return launch_nt<P, 128, 128, TOut>(g, s);
  return launch_nt<P, 64, 64, TOut>(g, s);
}

template <int P>
static hipError_t dispatch_out(int c_dtype, const GemmArgs& g, hipStream_t s) {
  switch (c_dtype) {
    case D_F64: return dispatch_nt<P, double>(g, s);
    case D_F32: return dispatch_nt<P, float>(g, s);
    case D_BF16: return dispatch_nt<P, bf16_t>(g, s);
  }
  return hipErrorInvalidValue;
}

hipError_t gemm_nt(int prec, int c_dtype, const GemmArgs& g, hipStream_t s) {
  switch (prec) {
    case P_F64: return dispatch_out<P_F64>(c_dtype, g, s);
    case P_F32: return dispatch_out<P_F32>(c_dtype, g, s);
    case P_BF16: return dispatch_out<P_BF16>(c_dtype, g, s);
  }
  return hipErrorInvalidValue;
}

template <int P, int BM, int BN, typename TOut>
static hipError_t launch_grouped(const GBases* bases, const GProb* probs, const GSeg* segs,
                                 const GTile* tiles, int64_t ntiles, int64_t a_bs, int64_t b_bs,
                                 int64_t c_bs, int nbatch, int max_wg, hipStream_t s) {
  using Cfg = TileCfg<P, BM, BN>;
  if (ntiles == 0 || nbatch == 0) return hipSuccess;
  int64_t g = ntiles;
  if (max_wg > 0 && g > max_wg) g = max_wg;
  dim3 grid((unsigned)g, (unsigned)nbatch);
  static const hipError_t attr = allow_lds(gemm_grouped_kernel<P, BM, BN, TOut>, Cfg::LDS_BYTES);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL((gemm_grouped_kernel<P, BM, BN, TOut>), grid, dim3(GEMM_THREADS),
                     Cfg::LDS_BYTES, s, bases, probs, segs, tiles, ntiles, a_bs, b_bs, c_bs);
  return hipGetLastError();
}

template <int P, int BM, int BN, int WM, int WN, typename TOut>
static hipError_t launch_grouped_direct(const GBases* bases, const GProb* probs, const GSeg* segs,
                                        const GTile* tiles, int64_t ntiles, int64_t a_bs, int64_t b_bs,
                                        int64_t c_bs, int nbatch, int max_wg, hipStream_t s) {
  using Cfg = DirectCfg<P, BM, BN, WM, WN>;
  if (ntiles == 0 || nbatch == 0) return hipSuccess;
  int64_t g = ntiles;
  if (max_wg > 0 && g > max_wg) g = max_wg;
  dim3 grid((unsigned)g, (unsigned)nbatch);
  constexpr int main_lds = Cfg::LDS_BYTES;
  constexpr int lds = sizeof(TOut) == 2 && epi_bytes<BM, BN>() > main_lds ? epi_bytes<BM, BN>() : main_lds;
  static const hipError_t attr = allow_lds(gemm_grouped_direct_kernel<P, BM, BN, WM, WN, TOut>, lds);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL((gemm_grouped_direct_kernel<P, BM, BN, WM, WN, TOut>), grid, dim3(Cfg::THREADS),
                     lds, s, bases, probs, segs, tiles, ntiles, a_bs, b_bs, c_bs);
  return hipGetLastError();
}

#define ITN_GROUPED_ARGS bases, probs, segs, tiles, ntiles, a_bs, b_bs, c_bs, nbatch, max_wg, s

template <int P, typename TOut>
static hipError_t grouped_cfg(int cfg, const GBases* bases, const GProb* probs, const GSeg* segs,
                              const GTile* tiles, int64_t ntiles, int64_t a_bs, int64_t b_bs,
                              int64_t c_bs, int nbatch, int max_wg, hipStream_t s) {
  if (cfg == 2) {
    if constexpr (P == P_F64) return launch_grouped_direct<P, 256, 128, 2, 4, TOut>(ITN_GROUPED_ARGS);
    else return launch_grouped_direct<P, 256, 256, 2, 4, TOut>(ITN_GROUPED_ARGS);
  }
  if (cfg == 3) return launch_grouped_direct<P, 128, 128, 2, 2, TOut>(ITN_GROUPED_ARGS);
  if (cfg == 4) return launch_grouped_direct<P, 256, 64, 4, 1, TOut>(ITN_GROUPED_ARGS);
  if (cfg == 1) return launch_grouped<P, 128, 128, TOut>(ITN_GROUPED_ARGS);
  return launch_grouped<P, 64, 64, TOut>(ITN_GROUPED_ARGS);
}

template <int P>
static hipError_t grouped_out(int c_dtype, int cfg, const GBases* bases, const GProb* probs,
                              const GSeg* segs, const GTile* tiles, int64_t ntiles, int64_t a_bs,
                              int64_t b_bs, int64_t c_bs, int nbatch, int max_wg, hipStream_t s) {
  switch (c_dtype) {
    case D_F64: return grouped_cfg<P, double>(cfg, ITN_GROUPED_ARGS);
    case D_F32: return grouped_cfg<P, float>(cfg, ITN_GROUPED_ARGS);
    case D_BF16: return grouped_cfg<P, bf16_t>(cfg, ITN_GROUPED_ARGS);
  }
  return hipErrorInvalidValue;
}

hipError_t gemm_grouped(int prec, int c_dtype, int tile_cfg, const GBases* bases, const GProb* probs,
                        const GSeg* segs, const GTile* tiles, int64_t ntiles, int64_t a_bs,
                        int64_t b_bs, int64_t c_bs, int nbatch, int max_wg, hipStream_t s) {
  const int cfg = tile_cfg;
  switch (prec) {
    case P_F64: return grouped_out<P_F64>(c_dtype, cfg, ITN_GROUPED_ARGS);
    case P_F32: return grouped_out<P_F32>(c_dtype, cfg, ITN_GROUPED_ARGS);
    case P_BF16: return grouped_out<P_BF16>(c_dtype, cfg, ITN_GROUPED_ARGS);
  }
  return hipErrorInvalidValue;
}
#undef ITN_GROUPED_ARGS

int grouped_tile_rows(int tile_cfg) {
  return (tile_cfg == 2 || tile_cfg == 4) ? 256 : (tile_cfg == 1 || tile_cfg == 3) ? 128 : 64;
}
int grouped_tile_cols(int prec, int tile_cfg) {
  if (tile_cfg == 2) return prec == P_F64 ? 128 : 256;
  if (tile_cfg == 4) return 64;
  return grouped_tile_rows(tile_cfg);
}

}  // namespace itn
