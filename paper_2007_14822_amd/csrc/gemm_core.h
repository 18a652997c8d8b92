// MFMA tile engine shared by the GEMM-shaped kernels of libitn.
//
// One workgroup of 256 threads (four wave64s in a 2x2 grid) computes a
// BM x BN tile of C = A * B^T, where both operands are K-contiguous rows
// ("NT").  K advances in steps of 128 bytes (16 f64 / 32 f32 / 64 bf16
// elements) through a double-buffered LDS stage; each LDS row is padded to
// 144 bytes so that the 16-byte fragment reads of 16 consecutive rows fall
// in distinct banks.  Every lane reads 16-byte fragments and feeds 16x16
// MFMAs: for bf16 one v_mfma_f32_16x16x32_bf16 per fragment pair, for f32
// four v_mfma_f32_16x16x4_f32, for f64 two v_mfma_f64_16x16x4_f64.  The
// K index order inside a step is a fixed permutation shared by A and B, so
// the sum is the plain sum over K.
#pragma once

#include "common.h"

namespace itn {

constexpr int GEMM_THREADS = 256;
constexpr int ROW_BYTES = 128;
constexpr int LDS_STRIDE = 144;

template <int P, int BM, int BN> struct TileCfg {
  using T = typename PT<P>::T;
  using Acc = typename PT<P>::Acc;
  using AccV = typename PT<P>::AccV;
  static constexpr int E16 = PT<P>::E16;
  static constexpr int BK = ROW_BYTES / (int)sizeof(T);
  static constexpr int FM = BM / 32;  // 16-row blocks per wave (two waves along M)
  static constexpr int FN = BN / 32;
  static constexpr int A_PASSES = BM / 32;  // 32 rows x 8 chunks per pass of 256 threads
  static constexpr int B_PASSES = BN / 32;
  static constexpr int STAGE_BYTES = (BM + BN) * LDS_STRIDE;
  static constexpr int LDS_BYTES = 2 * STAGE_BYTES;
};

template <typename T> __device__ __forceinline__ T zero_of() { return (T)0.0f; }

// 16 bytes of row `row` starting at element k; zero outside [0, nrows) x [0, K).
template <typename T, int E16, bool ALIGNED>
__device__ __forceinline__ uint4 load16(const T* __restrict__ base, int64_t ld, int64_t row,
                                        int64_t nrows, int64_t k, int64_t K) {
  uint4 v = {0u, 0u, 0u, 0u};
  if (row < nrows) {
    const T* p = base + row * ld + k;
    if (ALIGNED && k + E16 <= K) {
      v = *reinterpret_cast<const uint4*>(p);
    } else {
      T tmp[E16];
#pragma unroll
      for (int e = 0; e < E16; ++e) tmp[e] = (k + e < K) ? p[e] : zero_of<T>();
      __builtin_memcpy(&v, tmp, 16);
    }
  }
  return v;
}

template <int P> struct Mfma;
template <> struct Mfma<P_BF16> {
  static __device__ __forceinline__ void run(const uint4& a, const uint4& b, floatx4& c) {
    bf16x8 av, bv;
    __builtin_memcpy(&av, &a, 16);
    __builtin_memcpy(&bv, &b, 16);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
  }
};
template <> struct Mfma<P_F32> {
  static __device__ __forceinline__ void run(const uint4& a, const uint4& b, floatx4& c) {
    float av[4], bv[4];
    __builtin_memcpy(av, &a, 16);
    __builtin_memcpy(bv, &b, 16);
#pragma unroll
    for (int e = 0; e < 4; ++e) c = __builtin_amdgcn_mfma_f32_16x16x4f32(av[e], bv[e], c, 0, 0, 0);
  }
};
template <> struct Mfma<P_F64> {
  static __device__ __forceinline__ void run(const uint4& a, const uint4& b, doublex4& c) {
    double av[2], bv[2];
    __builtin_memcpy(av, &a, 16);
    __builtin_memcpy(bv, &b, 16);
#pragma unroll
    for (int e = 0; e < 2; ++e) c = __builtin_amdgcn_mfma_f64_16x16x4f64(av[e], bv[e], c, 0, 0, 0);
  }
};

template <int P, int BM, int BN>
__device__ __forceinline__ void zero_acc(typename TileCfg<P, BM, BN>::AccV (&acc)[BM / 32][BN / 32]) {
#pragma unroll
  for (int i = 0; i < BM / 32; ++i)
#pragma unroll
    for (int j = 0; j < BN / 32; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[i][j][e] = 0;
}

// acc += A[m0:m0+BM, 0:K] * B[n0:n0+BN, 0:K]^T.  A and B point at row 0 of
// their operand; rows >= M (resp. N) and k >= K read as zero.  Ends with a
// barrier, so it may be called again on the same LDS.
template <int P, int BM, int BN, bool ALIGNED>
__device__ __forceinline__ void gemm_accum(
    const typename PT<P>::T* __restrict__ A, int64_t lda, int64_t M,
    const typename PT<P>::T* __restrict__ B, int64_t ldb, int64_t N, int64_t K, int64_t m0,
    int64_t n0, typename TileCfg<P, BM, BN>::AccV (&acc)[BM / 32][BN / 32], char* lds) {
  using C = TileCfg<P, BM, BN>;
  using T = typename C::T;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lrow = tid >> 3, lchunk = tid & 7;
  const int q = lane >> 4, r16 = lane & 15;
  const int64_t nk = (K + C::BK - 1) / C::BK;
  if (nk <= 0) return;
  uint4 ra[C::A_PASSES], rb[C::B_PASSES];

  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int p = 0; p < C::A_PASSES; ++p)
      ra[p] = load16<T, C::E16, ALIGNED>(A, lda, m0 + p * 32 + lrow, M, k0 + lchunk * C::E16, K);
#pragma unroll
    for (int p = 0; p < C::B_PASSES; ++p)
      rb[p] = load16<T, C::E16, ALIGNED>(B, ldb, n0 + p * 32 + lrow, N, k0 + lchunk * C::E16, K);
  };
  auto sstore = [&](int buf) {
    char* a = lds + buf * C::STAGE_BYTES;
    char* b = a + BM * LDS_STRIDE;
#pragma unroll
    for (int p = 0; p < C::A_PASSES; ++p)
      *reinterpret_cast<uint4*>(a + (p * 32 + lrow) * LDS_STRIDE + lchunk * 16) = ra[p];
#pragma unroll
    for (int p = 0; p < C::B_PASSES; ++p)
      *reinterpret_cast<uint4*>(b + (p * 32 + lrow) * LDS_STRIDE + lchunk * 16) = rb[p];
  };

  gload(0);
  sstore(0);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = (int)(kt & 1);
    if (kt + 1 < nk) gload((kt + 1) * C::BK);
    const char* As = lds + cur * C::STAGE_BYTES;
    const char* Bs = As + BM * LDS_STRIDE;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      uint4 af[C::FM], bfr[C::FN];
#pragma unroll
      for (int i = 0; i < C::FM; ++i)
        af[i] = *reinterpret_cast<const uint4*>(As + (wm * (BM / 2) + i * 16 + r16) * LDS_STRIDE +
                                                ks * 64 + q * 16);
#pragma unroll
      for (int j = 0; j < C::FN; ++j)
        bfr[j] = *reinterpret_cast<const uint4*>(Bs + (wn * (BN / 2) + j * 16 + r16) * LDS_STRIDE +
                                                 ks * 64 + q * 16);
#pragma unroll
      for (int i = 0; i < C::FM; ++i)
#pragma unroll
        for (int j = 0; j < C::FN; ++j) Mfma<P>::run(af[i], bfr[j], acc[i][j]);
    }
    if (kt + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Direct-to-LDS variant.  gfx950's global_load_lds_dwordx4 writes the 16
// bytes each lane loads straight into LDS, lane i at (wave-uniform base +
// 16*i), so no registers stage the tiles.  One wave fills 8 rows x 128 bytes
// per instruction; LDS rows are 128 bytes wide and their eight 16-byte chunks
// are XOR-swizzled by (row % 8), which keeps the fragment reads of 8
// consecutive rows in distinct banks.  The chunk a lane writes is fixed by
// its lane id, so the swizzle is applied by choosing which global chunk the
// lane loads.  Requires 16-byte aligned rows and K % BK == 0; rows past M
// (or N) are clamped to the last row (their results are never stored).

__device__ __forceinline__ void lds_direct16(const void* g, void* lds_wave_base) {
  __builtin_amdgcn_global_load_lds(
      (const __attribute__((address_space(1))) void*)g,
      (__attribute__((address_space(3))) void*)lds_wave_base, 16, 0, 0);
}

template <int P, int BM, int BN, int WM, int WN> struct DirectCfg {
  using T = typename PT<P>::T;
  using AccV = typename PT<P>::AccV;
  static constexpr int THREADS = 64 * WM * WN;
  static constexpr int NW = WM * WN;
  static constexpr int E16 = PT<P>::E16;
  static constexpr int BK = ROW_BYTES / (int)sizeof(T);
  static constexpr int TM = BM / WM, TN = BN / WN;  // wave tile
  static constexpr int FM = TM / 16, FN = TN / 16;
  static constexpr int STAGE_BYTES = (BM + BN) * ROW_BYTES;
  static constexpr int LDS_BYTES = 2 * STAGE_BYTES;
  static constexpr int ROWS_PER_PASS = 8 * NW;
  static constexpr int A_PASSES = BM / ROWS_PER_PASS;
  static constexpr int B_PASSES = BN / ROWS_PER_PASS;
  static_assert(BM % ROWS_PER_PASS == 0 && BN % ROWS_PER_PASS == 0, "tile vs waves");
};

// acc += A[m0:m0+BM, 0:K] * B[n0:n0+BN, 0:K]^T with direct-to-LDS staging.
// Without KTAIL, K is a whole number of K steps.  With KTAIL, K may end
// inside a step: rows must be readable (and zero) up to K rounded up to 16
// bytes, and 16-byte chunks beyond that are loaded from `zero` (at least 16
// zero bytes) instead of the row.
template <int P, int BM, int BN, int WM, int WN, bool KTAIL = false>
__device__ __forceinline__ void gemm_accum_direct(
    const typename PT<P>::T* __restrict__ A, int64_t lda, int64_t M,
    const typename PT<P>::T* __restrict__ B, int64_t ldb, int64_t N, int64_t K, int64_t m0,
    int64_t n0,
    typename PT<P>::AccV (&acc)[DirectCfg<P, BM, BN, WM, WN>::FM][DirectCfg<P, BM, BN, WM, WN>::FN],
    char* lds, const typename PT<P>::T* zero = nullptr) {
  using C = DirectCfg<P, BM, BN, WM, WN>;
  using T = typename C::T;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int q = lane >> 4, r16 = lane & 15;
  const int64_t nk = KTAIL ? (K + C::BK - 1) / C::BK : K / C::BK;
  if (nk <= 0) return;
  const int64_t kpad = (K + C::E16 - 1) / C::E16 * C::E16;  // readable row length
  const int lrow = lane >> 3;  // row within the wave's 8-row slab
  const int lpos = lane & 7;   // LDS chunk slot this lane fills
  const int slab = wave * 8 + lrow;
  // The swizzle (lpos ^ row%8) only depends on lrow since slab starts are multiples of 8.
  const int64_t chunk = (int64_t)((lpos ^ lrow) * C::E16);
  const bool fullA = m0 + BM <= M, fullB = n0 + BN <= N;
  auto rowA = [&](int p) -> const T* {
    int64_t gr = m0 + p * C::ROWS_PER_PASS + slab;
    if (!fullA && gr >= M) gr = M - 1;
    return A + gr * lda + chunk;
  };
  auto rowB = [&](int p) -> const T* {
    int64_t gr = n0 + p * C::ROWS_PER_PASS + slab;
    if (!fullB && gr >= N) gr = N - 1;
    return B + gr * ldb + chunk;
  };
  auto issue = [&](char* __restrict__ stage, int64_t k0) {
    char* a = stage + wave * 8 * ROW_BYTES;
    char* b = stage + BM * ROW_BYTES + wave * 8 * ROW_BYTES;
    // with KTAIL, chunks past the row's readable length come from the zero page
    const bool tail = KTAIL && k0 + chunk >= kpad;
#pragma unroll
    for (int p = 0; p < C::A_PASSES; ++p)
      lds_direct16(tail ? zero : rowA(p) + k0, a + p * C::ROWS_PER_PASS * ROW_BYTES);
#pragma unroll
    for (int p = 0; p < C::B_PASSES; ++p)
      lds_direct16(tail ? zero : rowB(p) + k0, b + p * C::ROWS_PER_PASS * ROW_BYTES);
  };
  // One K step: the direct loads of the next stage into `nxt` overlap the
  // MFMAs on `cur`.  The stages never alias; the restrict-qualified
  // parameters let the compiler see that, so it does not wait for the
  // loads before its LDS reads of `cur` (the wait at the end of the step
  // is explicit).
  auto kstep = [&](const char* __restrict__ cur, char* __restrict__ nxt, bool more, int64_t k0) {
    if (more) issue(nxt, k0);
    const char* As = cur;
    const char* Bs = As + BM * ROW_BYTES;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int c = ks * 4 + q;
      uint4 bfr[C::FN];
#pragma unroll
      for (int j = 0; j < C::FN; ++j) {
        const int R = wn * C::TN + j * 16 + r16;
        bfr[j] = *reinterpret_cast<const uint4*>(Bs + R * ROW_BYTES + ((c ^ (R & 7)) << 4));
      }
#pragma unroll
      for (int i = 0; i < C::FM; ++i) {
        const int R = wm * C::TM + i * 16 + r16;
        const uint4 af = *reinterpret_cast<const uint4*>(As + R * ROW_BYTES + ((c ^ (R & 7)) << 4));
#pragma unroll
        for (int j = 0; j < C::FN; ++j) Mfma<P>::run(af, bfr[j], acc[i][j]);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of the next tile have landed in LDS
    __syncthreads();
  };

  issue(lds, 0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = (int)(kt & 1);
    kstep(lds + cur * C::STAGE_BYTES, lds + (cur ^ 1) * C::STAGE_BYTES, kt + 1 < nk,
          (kt + 1) * C::BK);
  }
}

// Store the wave's FM x FN accumulator blocks of a direct tile.
// MODE: 0 store, 1 accumulate into C, 2 store with nontemporal hints (C is
// consumed by a later pass, not by the next kernel's cache-resident reads).
template <int P, int BM, int BN, int WM, int WN, typename TOut, int MODE>
__device__ __forceinline__ void store_tile_direct(
    const typename PT<P>::AccV (&acc)[DirectCfg<P, BM, BN, WM, WN>::FM][DirectCfg<P, BM, BN, WM, WN>::FN],
    TOut* __restrict__ Cp, int64_t ldc, int64_t M, int64_t N, int64_t m0, int64_t n0,
    const int64_t* __restrict__ rows = nullptr) {
  using C = DirectCfg<P, BM, BN, WM, WN>;
  using Acc = typename PT<P>::Acc;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const bool full = m0 + BM <= M && n0 + BN <= N;
#pragma unroll
  for (int i = 0; i < C::FM; ++i)
#pragma unroll
    for (int j = 0; j < C::FN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = m0 + wm * C::TM + i * 16 + acc_row<P>(lane, e);
        const int64_t col = n0 + wn * C::TN + j * 16 + (lane & 15);
        if (full || (row < M && col < N)) {
          Acc v = acc[i][j][e];
          TOut* p = Cp + (rows ? rows[row] : row * ldc) + col;
          if constexpr (MODE == 1) {
            v += cvt<Acc>(*p);
            *p = cvt<TOut>(v);
          } else if constexpr (MODE == 2) {
            __builtin_nontemporal_store(cvt<TOut>(v), p);
          } else {
            *p = cvt<TOut>(v);
          }
        }
      }
}

// Store of a 2-byte direct tile through LDS: the accumulators are converted
// into an LDS copy of the tile (rows padded by 16 bytes so that the four
// row groups of a lane's column start in different banks), then every
// thread writes whole 16-byte vectors of a row, so each row of the tile
// leaves as one contiguous run instead of 32-byte pieces from several
// waves.  Needs C rows 16-byte aligned (C, ldc and the column origin
// multiples of 8) and N a multiple of 8; `lds` holds at least
// EpiBytes<BM, BN> bytes and is free on entry and on return.  STREAM:
// nontemporal stores (C is read once by a later pass and does not fit the
// caches; the stores then do not displace the operands' lines).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <int BM, int BN> constexpr int epi_bytes() { return BM * (BN + 8) * 2; }
template <int P, int BM, int BN, int WM, int WN, typename TOut, bool STREAM>
__device__ __forceinline__ void store_tile_lds(
    const typename PT<P>::AccV (&acc)[DirectCfg<P, BM, BN, WM, WN>::FM][DirectCfg<P, BM, BN, WM, WN>::FN],
    TOut* __restrict__ Cp, int64_t ldc, int64_t M, int64_t N, int64_t m0, int64_t n0, char* lds) {
  static_assert(sizeof(TOut) == 2, "2-byte outputs only");
  using C = DirectCfg<P, BM, BN, WM, WN>;
  constexpr int LD = BN + 8;
  TOut* t = reinterpret_cast<TOut*>(lds);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  __syncthreads();  // every wave is done with the K loop's LDS stages
#pragma unroll
  for (int i = 0; i < C::FM; ++i)
#pragma unroll
    for (int j = 0; j < C::FN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = wm * C::TM + i * 16 + acc_row<P>(lane, e);
        const int col = wn * C::TN + j * 16 + (lane & 15);
        t[row * LD + col] = cvt<TOut>(acc[i][j][e]);
      }
  __syncthreads();
  constexpr int VPR = BN / 8;               // 16-byte vectors per tile row
  constexpr int RPP = C::THREADS / VPR;     // rows per pass
  static_assert(C::THREADS % VPR == 0 && BM % RPP == 0, "epilogue passes");
  const int rr = tid / VPR, cv = (tid % VPR) * 8;
  const int64_t gc = n0 + cv;
#pragma unroll 4
  for (int r0 = 0; r0 < BM; r0 += RPP) {
    const int r = r0 + rr;
    const int64_t gr = m0 + r;
    if (gr < M && gc < N) {
      const u32x4 v = *reinterpret_cast<const u32x4*>(t + r * LD + cv);
      u32x4* dst = reinterpret_cast<u32x4*>(Cp + gr * ldc + gc);
      if constexpr (STREAM) __builtin_nontemporal_store(v, dst);
      else *dst = v;
    }
  }
  __syncthreads();  // the next tile's loads overwrite the LDS
}

// Write (or add to) the BM x BN tile at (m0, n0) of C (rows >= M or cols >= N skipped).
template <int P, int BM, int BN, typename TOut>
__device__ __forceinline__ void store_tile(
    const typename TileCfg<P, BM, BN>::AccV (&acc)[BM / 32][BN / 32], TOut* __restrict__ Cp,
    int64_t ldc, int64_t M, int64_t N, int64_t m0, int64_t n0, bool accumulate,
    const int64_t* __restrict__ rows = nullptr) {
  using Acc = typename PT<P>::Acc;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
#pragma unroll
  for (int i = 0; i < BM / 32; ++i)
#pragma unroll
    for (int j = 0; j < BN / 32; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = m0 + wm * (BM / 2) + i * 16 + acc_row<P>(lane, e);
        const int64_t col = n0 + wn * (BN / 2) + j * 16 + (lane & 15);
        if (row < M && col < N) {
          Acc v = acc[i][j][e];
          TOut* p = Cp + (rows ? rows[row] : row * ldc) + col;
          if (accumulate) v += cvt<Acc>(*p);
          *p = cvt<TOut>(v);
        }
      }
}

// Tile order: spread consecutive logical tiles over the 8 XCDs' own
// dispatch slots (workgroup i runs on XCD i % 8), then walk tiles in groups
// of 8 tile-rows so that tiles resident on one XCD share A and B panels.
__device__ __forceinline__ void tile_coords(int64_t bid, int64_t ntiles, int64_t tiles_m,
                                            int64_t tiles_n, int64_t& tm, int64_t& tn) {
  int64_t logical = bid;
  const int64_t per = ntiles / 8;
  if (per > 0 && bid < per * 8) logical = (bid % 8) * per + bid / 8;
  const int64_t G = 8;
  const int64_t width = G * tiles_n;
  const int64_t group = logical / width;
  const int64_t first_m = group * G;
  int64_t gsize = tiles_m - first_m;
  if (gsize > G) gsize = G;
  const int64_t in_group = logical % width;
  tm = first_m + in_group % gsize;
  tn = in_group / gsize;
}

}  // namespace itn
