// Fused first stage of the dense two-site H_eff:
//
//   X[a', m0, c, y] = sum_a L[a', m0, a] psiT[c, y, a]          (MFMA)
//   Z[v, a', c', m2, b] = sum_{m0, c} W12[(c', m2), (m0, c)] X[a', m0, c, y]   (epilogue)
//
// with c = (s1, s2), y = (v, b), W12 = sum_m1 W1 W2 (sparse, CSR by output).
// The tile of one workgroup covers a block of a' and a block of y for *all*
// (m0, c) pairs: its A rows are (m0, a') and its B rows (c, y), and every
// wave owns complete (m0, c) sets for its 16 x 16 (a', y) sub-blocks, so the
// MFMA accumulators of one lane hold every X value its positions need.  The
// epilogue writes them to a per-wave LDS area (input-major, lane-minor, so
// that the gather below is bank-conflict free), then applies W12 row by row
// from a CSR table and writes Z straight to HBM.  X never leaves the chip.
// The CSR table (at most 63 rows and 128 entries) is loaded into lane
// registers when the kernel starts, under the main loop, and read back
// with readlane: the epilogue issues no memory loads besides its LDS
// gathers.
#include "gemm_core.h"
#include "kernels.h"

namespace itn {

// Raw buffer descriptor over [base, base + bytes) (bytes < 2^31); the third
// descriptor word selects 32-bit data for untyped buffer loads.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
// 16 bytes per lane from base + voff + soff into LDS at lds_wave_base + 16 * lane.
__device__ __forceinline__ void lds_buffer16(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff,
                                             void* lds_wave_base) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)lds_wave_base, 16,
                                           voff, soff, 0, 0);
}

template <int P, int W, int C, int WM, int WN, int RA, int RB> struct FusedCfg {
  using T = typename PT<P>::T;
  using Acc = typename PT<P>::Acc;
  using AccV = typename PT<P>::AccV;
  static constexpr int NW = WM * WN;
  static constexpr int THREADS = 64 * NW;
  static constexpr int E16 = PT<P>::E16;
  static constexpr int BK = ROW_BYTES / (int)sizeof(T);
  static constexpr int TA = WM * 16 * RA;  // a' per workgroup
  static constexpr int TY = WN * 16 * RB;  // y per workgroup
  static constexpr int AROWS = W * TA;
  static constexpr int BROWS = C * TY;
  static constexpr int STAGE_BYTES = (AROWS + BROWS) * ROW_BYTES;
  static constexpr int RPP = 8 * NW;  // rows per direct-load pass
  static constexpr int A_PASSES = (AROWS + RPP - 1) / RPP;
  static constexpr int B_PASSES = (BROWS + RPP - 1) / RPP;
  // Epilogue: GP position groups per pass, stored interleaved as
  // [input (m0, c)][lane][group] so that a lane writes and gathers GP values
  // with one LDS instruction.
  static constexpr int GROUPS = RA * RB * 4;
  static constexpr int LDS_MAX = 163840;
  static constexpr int GP_BYTES1 = NW * W * C * 64 * (int)sizeof(Acc);
  static constexpr int GP = (GROUPS % 4 == 0 && 4 * GP_BYTES1 <= LDS_MAX) ? 4
                          : (GROUPS % 2 == 0 && 2 * GP_BYTES1 <= LDS_MAX) ? 2 : 1;
  static constexpr int EPI_BYTES = GP * GP_BYTES1;
  static constexpr int LDS_BYTES = (2 * STAGE_BYTES > EPI_BYTES) ? 2 * STAGE_BYTES : EPI_BYTES;
  static_assert(LDS_BYTES <= LDS_MAX, "LDS budget");
};

template <int P, int W, int C, int WM, int WN, int RA, int RB, typename TZ>
__global__ __launch_bounds__(64 * WM * WN) void heff_fused_kernel(HeffFusedArgs a, int64_t tiles_a,
                                                                   int64_t tiles_y) {
  using Cfg = FusedCfg<P, W, C, WM, WN, RA, RB>;
  using T = typename Cfg::T;
  using Acc = typename Cfg::Acc;
  extern __shared__ __align__(16) char lds[];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int q = lane >> 4, r16 = lane & 15;
  int64_t ta, ty;
  tile_coords(blockIdx.x, tiles_a * tiles_y, tiles_a, tiles_y, ta, ty);
  const int64_t a0 = ta * Cfg::TA, y0 = ty * Cfg::TY;
  const int64_t cl = a.chi_l, Y = (int64_t)a.nv * a.chi_r;
  const T* Lp = static_cast<const T*>(a.L);
  const T* Bp = static_cast<const T*>(a.psiT);
  const int64_t nk = cl / Cfg::BK;

  // W12 table in lane registers: lane l holds row_ptr[l] and entries l and
  // 64 + l (LDS byte offset of the gathered input and coefficient).
  constexpr int GP = Cfg::GP;
  constexpr int IN_BYTES = 64 * GP * (int)sizeof(Acc);  // LDS bytes per input
  const int tab_rp = lane <= a.nrows ? a.row_ptr[lane] : 0;
  int tab_off[2];
  Acc tab_cf[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int e = h * 64 + lane;
    const bool in = e < a.nnz;
    tab_off[h] = in ? a.col_idx[e] * IN_BYTES : 0;
    tab_cf[h] = in ? ((P == P_F64) ? (Acc)a.coef64[e] : (Acc)a.coef32[e]) : (Acc)0;
  }

  typename Cfg::AccV acc[W][RA][C][RB];
#pragma unroll
  for (int m = 0; m < W; ++m)
#pragma unroll
    for (int i = 0; i < RA; ++i)
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int j = 0; j < RB; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[m][i][c][j][e] = 0;

  // Direct-to-LDS row sources (see gemm_core.h for the swizzle), through
  // buffer descriptors: uniform 64-bit bases, one 32-bit lane offset per
  // operand, and per pass a uniform byte offset.  Tile row r = p*RPP + slab
  // of A is (m0, a') = (r / TA, a0 + r % TA); RPP is a multiple of TA and
  // of TY, so the lane part of the row (r % TA, r / TA - p*RPP/TA) is the
  // same in every pass and the pass adds p*(RPP/TA) rows of m0 (likewise
  // for B's (c, y)).  Both operands are below 2^31 bytes (checked by the
  // launcher).  Rows beyond chi_l (or Y) are clamped to the last row.
  static_assert(Cfg::RPP % Cfg::TA == 0 && Cfg::RPP % Cfg::TY == 0, "pass stride vs tile rows");
  const int lrow = lane >> 3, lpos = lane & 7;
  const int slab = wave * 8 + lrow;
  const int64_t chunk = (int64_t)((lpos ^ lrow) * Cfg::E16);
  constexpr int ES = (int)sizeof(T);
  const __amdgpu_buffer_rsrc_t rsA = make_rsrc(Lp, cl * W * cl * ES);
  const __amdgpu_buffer_rsrc_t rsB = make_rsrc(Bp, (int64_t)C * Y * cl * ES);
  uint32_t voffA, voffB;
  {
    int64_t ap = a0 + slab % Cfg::TA;
    if (ap >= cl) ap = cl - 1;
    voffA = (uint32_t)(((ap * W + slab / Cfg::TA) * cl + chunk) * ES);
    int64_t y = y0 + slab % Cfg::TY;
    if (y >= Y) y = Y - 1;
    voffB = (uint32_t)((((int64_t)(slab / Cfg::TY) * Y + y) * cl + chunk) * ES);
  }
  const uint32_t passA = (uint32_t)((Cfg::RPP / Cfg::TA) * cl * ES);      // one pass: RPP/TA more m0
  const uint32_t passB = (uint32_t)((Cfg::RPP / Cfg::TY) * Y * cl * ES);  // RPP/TY more c
  auto issue = [&](int buf, int64_t k0) {
    char* base = lds + buf * Cfg::STAGE_BYTES + wave * 8 * ROW_BYTES;
    const uint32_t kb = (uint32_t)(k0 * ES);
#pragma unroll
    for (int p = 0; p < Cfg::A_PASSES; ++p)
      if (p * Cfg::RPP + wave * 8 < Cfg::AROWS)
        lds_buffer16(rsA, voffA, p * passA + kb, base + p * Cfg::RPP * ROW_BYTES);
#pragma unroll
    for (int p = 0; p < Cfg::B_PASSES; ++p)
      if (p * Cfg::RPP + wave * 8 < Cfg::BROWS)
        lds_buffer16(rsB, voffB, p * passB + kb, base + (Cfg::AROWS + p * Cfg::RPP) * ROW_BYTES);
  };

  if (nk > 0) {
    issue(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  // One K step: direct loads of the next stage into `nxt` overlap the MFMAs
  // on `cur`.  The two stages never alias; restrict-qualified parameters let
  // the compiler see that and not wait for the loads before reading `cur`.
  auto kstep = [&](const char* __restrict__ cur, char* __restrict__ nxt, bool more, int64_t k0) {
    if (more) {
      char* base = nxt + wave * 8 * ROW_BYTES;
      const uint32_t kb = (uint32_t)(k0 * ES);
#pragma unroll
      for (int p = 0; p < Cfg::A_PASSES; ++p)
        if (p * Cfg::RPP + wave * 8 < Cfg::AROWS)
          lds_buffer16(rsA, voffA, p * passA + kb, base + p * Cfg::RPP * ROW_BYTES);
#pragma unroll
      for (int p = 0; p < Cfg::B_PASSES; ++p)
        if (p * Cfg::RPP + wave * 8 < Cfg::BROWS)
          lds_buffer16(rsB, voffB, p * passB + kb, base + (Cfg::AROWS + p * Cfg::RPP) * ROW_BYTES);
    }
    const char* As = cur;
    const char* Bs = As + Cfg::AROWS * ROW_BYTES;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int ch = ks * 4 + q;
      uint4 bfr[C][RB];
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int j = 0; j < RB; ++j) {
          const int R = c * Cfg::TY + wn * 16 * RB + j * 16 + r16;
          bfr[c][j] = *reinterpret_cast<const uint4*>(Bs + R * ROW_BYTES + ((ch ^ (R & 7)) << 4));
        }
#pragma unroll
      for (int m = 0; m < W; ++m)
#pragma unroll
        for (int i = 0; i < RA; ++i) {
          const int R = m * Cfg::TA + wm * 16 * RA + i * 16 + r16;
          const uint4 af = *reinterpret_cast<const uint4*>(As + R * ROW_BYTES + ((ch ^ (R & 7)) << 4));
#pragma unroll
          for (int c = 0; c < C; ++c)
#pragma unroll
            for (int j = 0; j < RB; ++j) Mfma<P>::run(af, bfr[c][j], acc[m][i][c][j]);
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  };
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = (int)(kt & 1);
    kstep(lds + cur * Cfg::STAGE_BYTES, lds + (cur ^ 1) * Cfg::STAGE_BYTES, kt + 1 < nk,
          (kt + 1) * Cfg::BK);
  }

  // ------------------------------------------------------------ W epilogue
  // The last K step ended with a barrier: the stage buffers are free.
  typedef Acc AccG __attribute__((ext_vector_type(GP)));
  char* ep = lds + wave * (W * C * IN_BYTES);
  const int64_t zs_v = cl * (int64_t)(C * W) * a.chi_r;  // Z stride of v
  const int64_t zs_a = (int64_t)(C * W) * a.chi_r;       // Z stride of a'
  TZ* Zp = static_cast<TZ*>(a.Z);
  // entry k of the table, broadcast from the lane that holds it
  auto entry = [&](int k, int& off, Acc& cf) {
    const int h = k >> 6, l = k & 63;
    const int ov = h ? tab_off[1] : tab_off[0];
    off = __builtin_amdgcn_readlane(ov, l);
    if constexpr (sizeof(Acc) == 8) {
      const double cv = h ? tab_cf[1] : tab_cf[0];
      const int64_t bits = __builtin_bit_cast(int64_t, cv);
      const int lo = __builtin_amdgcn_readlane((int)bits, l);
      const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
      cf = __builtin_bit_cast(double, ((int64_t)hi << 32) | (uint32_t)lo);
    } else {
      const float cv = h ? tab_cf[1] : tab_cf[0];
      cf = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, cv), l));
    }
  };
#pragma unroll
  for (int g0 = 0; g0 < Cfg::GROUPS; g0 += GP) {
    TZ* zrow[GP];
    bool ok[GP];
#pragma unroll
    for (int m = 0; m < W; ++m)
#pragma unroll
      for (int c = 0; c < C; ++c) {
        AccG v;
#pragma unroll
        for (int gg = 0; gg < GP; ++gg) {
          const int g = g0 + gg;
          v[gg] = acc[m][g / (RB * 4)][c][(g / 4) % RB][g % 4];
        }
        *reinterpret_cast<AccG*>(ep + (m * C + c) * IN_BYTES + lane * (GP * (int)sizeof(Acc))) = v;
      }
#pragma unroll
    for (int gg = 0; gg < GP; ++gg) {
      const int g = g0 + gg;
      const int i = g / (RB * 4), j = (g / 4) % RB, e = g % 4;
      const int64_t ap = a0 + wm * 16 * RA + i * 16 + acc_row<P>(lane, e);
      const int64_t y = y0 + wn * 16 * RB + j * 16 + (lane & 15);
      ok[gg] = ap < cl && y < Y;
      const int64_t vv = ok[gg] ? y / a.chi_r : 0, b = ok[gg] ? y % a.chi_r : 0;
      zrow[gg] = Zp + vv * zs_v + ap * zs_a + b;
    }
    // Each lane reads back only its own slots: no barrier needed.  All
    // W*C output rows are formed in registers first, then stored together.
    const char* mine = ep + lane * (GP * (int)sizeof(Acc));
    int k = __builtin_amdgcn_readlane(tab_rp, 0);
    AccG zz[W * C];
#pragma unroll
    for (int o = 0; o < W * C; ++o) {
      AccG z = (Acc)0;
      const int e1 = __builtin_amdgcn_readlane(tab_rp, o + 1);
      for (; k < e1; k += 2) {
        int o0, o1;
        Acc c0, c1;
        entry(k, o0, c0);
        entry(k + 1 < e1 ? k + 1 : k, o1, c1);
        if (k + 1 >= e1) c1 = (Acc)0;
        const AccG x0 = *reinterpret_cast<const AccG*>(mine + o0);
        const AccG x1 = *reinterpret_cast<const AccG*>(mine + o1);
        z += c0 * x0 + c1 * x1;
      }
      k = e1;
      zz[o] = z;
    }
#pragma unroll
    for (int o = 0; o < W * C; ++o)
#pragma unroll
      for (int gg = 0; gg < GP; ++gg)
        if (ok[gg]) zrow[gg][(int64_t)o * a.chi_r] = cvt<TZ>(zz[o][gg]);
  }
}

template <int P> struct FusedPick;  // configuration per precision and (w, d^2)

template <int P, int W, int C, int WM, int WN, int RA, int RB>
static hipError_t launch_fused(const HeffFusedArgs& a, hipStream_t s) {
  using Cfg = FusedCfg<P, W, C, WM, WN, RA, RB>;
  using T = typename Cfg::T;
  const int64_t Y = (int64_t)a.nv * a.chi_r;
  const int64_t tiles_a = (a.chi_l + Cfg::TA - 1) / Cfg::TA, tiles_y = (Y + Cfg::TY - 1) / Cfg::TY;
  if (tiles_a == 0 || tiles_y == 0) return hipSuccess;
  auto kern = heff_fused_kernel<P, W, C, WM, WN, RA, RB, T>;
  static const hipError_t attr =
      Cfg::LDS_BYTES > 65536
          ? hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize, Cfg::LDS_BYTES)
          : hipSuccess;
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(kern, dim3((unsigned)(tiles_a * tiles_y)), dim3(Cfg::THREADS),
                     Cfg::LDS_BYTES, s, a, tiles_a, tiles_y);
  return hipGetLastError();
}

bool heff_fused_supported(int prec, int w, int d2) {
  if (w < 3 || w > 5) return false;
  if (d2 == 4) return true;
  if (d2 == 9) return prec != P_F64;
  return false;
}

bool heff_fused_table_fits(int nrows, int64_t nnz) {
  return nrows >= 1 && nrows <= 63 && nnz >= 0 && nnz <= 128;  // lane-register table
}

template <int P, int W> static hipError_t fused_w(const HeffFusedArgs& a, hipStream_t s) {
  if constexpr (P == P_F64) {
    return launch_fused<P, W, 4, 2, 4, 1, 1>(a, s);
  } else {
    if (a.d2 == 4) return launch_fused<P, W, 4, 2, 4, 2, 1>(a, s);
    return launch_fused<P, W, 9, 4, 2, 1, 1>(a, s);
  }
}

template <int P> static hipError_t fused_p(const HeffFusedArgs& a, hipStream_t s) {
  switch (a.w) {
    case 3: return fused_w<P, 3>(a, s);
    case 4: return fused_w<P, 4>(a, s);
    case 5: return fused_w<P, 5>(a, s);
  }
  return hipErrorInvalidValue;
}

bool heff_fused_fits(int prec, int64_t chi_l, int64_t chi_r, int w, int d2, int nv) {
  const int64_t es = prec == P_F64 ? 8 : prec == P_F32 ? 4 : 2;
  const int64_t lim = (int64_t)1 << 31;  // buffer-descriptor range of each operand
  return chi_l * w * chi_l * es < lim && (int64_t)d2 * nv * chi_r * chi_l * es < lim;
}

hipError_t heff_stage1_fused(int prec, const HeffFusedArgs& a, hipStream_t s) {
  if (!heff_fused_supported(prec, a.w, a.d2)) return hipErrorInvalidValue;
  if (!heff_fused_fits(prec, a.chi_l, a.chi_r, a.w, a.d2, a.nv)) return hipErrorInvalidValue;
  // the epilogue unrolls over all w*d2 output rows of W12
  if (a.nrows != a.w * a.d2 || !heff_fused_table_fits(a.nrows, a.nnz)) return hipErrorInvalidValue;
  switch (prec) {
    case P_BF16: return fused_p<P_BF16>(a, s);
    case P_F32: return fused_p<P_F32>(a, s);
    case P_F64: return fused_p<P_F64>(a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace itn
