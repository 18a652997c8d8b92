// Memory-bound kernels of libitn: layout changes with dtype conversion, the
// sparse W-stage, and the FP64 vector operations of the eigensolver.
#include "common.h"
#include "kernels.h"

namespace itn {

// ------------------------------------------------------------------ helpers
template <typename T> struct DT;
template <> struct DT<double> { static constexpr int code = D_F64; };
template <> struct DT<float> { static constexpr int code = D_F32; };
template <> struct DT<bf16_t> { static constexpr int code = D_BF16; };

#define ITN_DISPATCH2(IN_DT, OUT_DT, FN, ...)                                         \
  do {                                                                                \
    if ((IN_DT) == D_F64 && (OUT_DT) == D_F64) return FN<double, double>(__VA_ARGS__);  \
    if ((IN_DT) == D_F64 && (OUT_DT) == D_F32) return FN<double, float>(__VA_ARGS__);   \
    if ((IN_DT) == D_F64 && (OUT_DT) == D_BF16) return FN<double, bf16_t>(__VA_ARGS__); \
    if ((IN_DT) == D_F32 && (OUT_DT) == D_F64) return FN<float, double>(__VA_ARGS__);   \
    if ((IN_DT) == D_F32 && (OUT_DT) == D_F32) return FN<float, float>(__VA_ARGS__);    \
    if ((IN_DT) == D_F32 && (OUT_DT) == D_BF16) return FN<float, bf16_t>(__VA_ARGS__);  \
    if ((IN_DT) == D_BF16 && (OUT_DT) == D_F64) return FN<bf16_t, double>(__VA_ARGS__); \
    if ((IN_DT) == D_BF16 && (OUT_DT) == D_F32) return FN<bf16_t, float>(__VA_ARGS__);  \
    if ((IN_DT) == D_BF16 && (OUT_DT) == D_BF16) return FN<bf16_t, bf16_t>(__VA_ARGS__);\
    return hipErrorInvalidValue;                                                      \
  } while (0)

template <typename To, typename From> __device__ __forceinline__ To conv(From x) {
  return (To)(float)x;
}
template <> __device__ __forceinline__ double conv<double, double>(double x) { return x; }
template <> __device__ __forceinline__ double conv<double, float>(float x) { return (double)x; }
template <> __device__ __forceinline__ float conv<float, double>(double x) { return (float)x; }
template <> __device__ __forceinline__ bf16_t conv<bf16_t, double>(double x) { return bf16_from_double(x); }

static unsigned grid_for(int64_t n, int threads, int64_t cap = 65536) {
  int64_t g = (n + threads - 1) / threads;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// -------------------------------------------------------------------- cast
template <typename TI, typename TO>
__global__ void cast_kernel(const TI* __restrict__ in, TO* __restrict__ out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = conv<TO, TI>(in[i]);
}
template <typename TI, typename TO>
static hipError_t cast_t(const void* in, void* out, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((cast_kernel<TI, TO>), dim3(grid_for(n, 256)), dim3(256), 0, s,
                     static_cast<const TI*>(in), static_cast<TO*>(out), n);
  return hipGetLastError();
}
hipError_t cast(int in_dtype, const void* in, int out_dtype, void* out, int64_t n, hipStream_t s) {
  ITN_DISPATCH2(in_dtype, out_dtype, cast_t, in, out, n, s);
}

// ----------------------------------------------------------------- permute
struct PermArgs {
  int rank;
  int64_t dims[8];
  int64_t istr[8];
  int64_t n;
};
template <typename TI, typename TO>
__global__ void permute_kernel(const TI* __restrict__ in, TO* __restrict__ out, PermArgs a) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = i, off = 0;
    for (int k = a.rank - 1; k >= 0; --k) {
      const int64_t c = rem % a.dims[k];
      rem /= a.dims[k];
      off += c * a.istr[k];
    }
    out[i] = conv<TO, TI>(in[off]);
  }
}
template <typename TI, typename TO>
static hipError_t permute_t(const void* in, void* out, const PermArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL((permute_kernel<TI, TO>), dim3(grid_for(a.n, 256)), dim3(256), 0, s,
                     static_cast<const TI*>(in), static_cast<TO*>(out), a);
  return hipGetLastError();
}
hipError_t permute_cast(int in_dtype, const void* in, int out_dtype, void* out, int rank,
                        const int64_t* out_dims, const int64_t* in_strides, hipStream_t s) {
  if (rank < 0 || rank > 8) return hipErrorInvalidValue;
  PermArgs a;
  a.rank = rank;
  a.n = 1;
  for (int k = 0; k < 8; ++k) {
    a.dims[k] = k < rank ? out_dims[k] : 1;
    a.istr[k] = k < rank ? in_strides[k] : 0;
    if (k < rank) a.n *= out_dims[k];
  }
  ITN_DISPATCH2(in_dtype, out_dtype, permute_t, in, out, a, s);
}

// ----------------------------------------------------------- permute batch
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void permute_batch_kernel(const TI* __restrict__ in,
                                                             TO* __restrict__ out,
                                                             const PermItem* __restrict__ items,
                                                             const PermChunk* __restrict__ chunks) {
  const PermChunk ch = chunks[blockIdx.x];
  const PermItem& it = items[ch.item];
  const int rank = it.rank;
  const int64_t end = ch.first + PERM_CHUNK < it.n ? ch.first + PERM_CHUNK : it.n;
  for (int64_t j = ch.first + threadIdx.x; j < end; j += blockDim.x) {
    int64_t rem = j, off = 0;
    for (int k = rank - 1; k >= 0; --k) {
      const int64_t c = rem % it.dims[k];
      rem /= it.dims[k];
      off += c * it.istr[k];
    }
    out[it.dst + j] = conv<TO, TI>(in[it.src + off]);
  }
}
template <typename TI, typename TO>
static hipError_t permute_batch_t(const void* in, void* out, const PermItem* items,
                                  const PermChunk* chunks, int64_t nchunks, hipStream_t s) {
  if (nchunks == 0) return hipSuccess;
  hipLaunchKernelGGL((permute_batch_kernel<TI, TO>), dim3((unsigned)nchunks), dim3(256), 0, s,
                     static_cast<const TI*>(in), static_cast<TO*>(out), items, chunks);
  return hipGetLastError();
}
hipError_t permute_batch(int in_dtype, const void* in, int out_dtype, void* out, const PermItem* items,
                         const PermChunk* chunks, int64_t nchunks, hipStream_t s) {
  ITN_DISPATCH2(in_dtype, out_dtype, permute_batch_t, in, out, items, chunks, nchunks, s);
}

__global__ __launch_bounds__(256) void copy2d_batch_kernel(const Copy2D* __restrict__ items,
                                                            const PermChunk* __restrict__ chunks) {
  const PermChunk ch = chunks[blockIdx.x];
  const Copy2D it = items[ch.item];
  const int64_t n = it.rows * it.cols;
  const int64_t end = ch.first + PERM_CHUNK < n ? ch.first + PERM_CHUNK : n;
  for (int64_t j = ch.first + threadIdx.x; j < end; j += blockDim.x) {
    const int64_t r = j / it.cols, c = j - r * it.cols;
    it.dst[r * it.ldd + c] = it.src[r * it.lds + c];
  }
}
hipError_t copy2d_batch(const Copy2D* items, const PermChunk* chunks, int64_t nchunks, hipStream_t s) {
  if (nchunks == 0) return hipSuccess;
  hipLaunchKernelGGL(copy2d_batch_kernel, dim3((unsigned)nchunks), dim3(256), 0, s, items, chunks);
  return hipGetLastError();
}

// --------------------------------------------------------------- transpose
// 64x64 tiles through LDS: coalesced reads along c, coalesced writes along r.
// Each element is converted once, as it is loaded, to the output type
// (FP64 -> bf16 is one rounding, not one to FP32 and another to bf16), and
// the tile holds the converted values: for the common FP64 -> bf16 case a
// quarter of the FP64 footprint, so more tiles stay resident.  Each lane
// writes two consecutive r of an output row.
constexpr int TT = 64;
template <typename TO> struct alignas(2 * sizeof(TO)) Pair { TO v[2]; };
template <typename TI> struct alignas(16) TW2 { TI v[2]; };
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void transpose_kernel(const TI* __restrict__ in,
                                                         TO* __restrict__ out, TransposeArgs t,
                                                         int64_t tiles_r, int64_t tiles_c) {
  __shared__ TO tile[TT][TT + 1];
  const int64_t z = blockIdx.y;
  const int64_t zb = z / t.nzc, zc = z % t.nzc;
  const int64_t tr = blockIdx.x / tiles_c, tc = blockIdx.x % tiles_c;
  const int64_t r0 = tr * TT, c0 = tc * TT;
  const TI* ip = in + zb * t.in_zb + zc * t.in_zc;
  TO* op = out + zb * t.out_zb + zc * t.out_zc;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
  using TW = typename std::conditional<sizeof(TI) == 8, double, float>::type;  // exact widening of TI
  // 8-byte inputs, unit stride along c, full tile, 16-byte aligned rows:
  // two consecutive c (16 bytes) per lane, 8 rows per pass.
  const bool wide_in = sizeof(TI) == 8 && t.in_c == 1 && r0 + TT <= t.rows && c0 + TT <= t.cols &&
                       (t.in_r % 2) == 0 && (reinterpret_cast<uintptr_t>(ip) % 16) == 0;
  if (wide_in) {
    const int c2 = (threadIdx.x & 31) * 2, ry = threadIdx.x >> 5;  // 32 pairs x 8 rows
#pragma unroll
    for (int i = ry; i < TT; i += 8) {
      const TW2<TI> v2 = *reinterpret_cast<const TW2<TI>*>(ip + (r0 + i) * t.in_r + c0 + c2);
      tile[i][c2] = conv<TO, TW>((TW)v2.v[0]);
      tile[i][c2 + 1] = conv<TO, TW>((TW)v2.v[1]);
    }
  } else {
#pragma unroll 4
    for (int i = ty; i < TT; i += 4) {
      const int64_t r = r0 + i, c = c0 + tx;
      if (r < t.rows && c < t.cols) tile[i][tx] = conv<TO, TW>((TW)ip[r * t.in_r + c * t.in_c]);
    }
  }
  __syncthreads();
  if constexpr (sizeof(TO) == 2) {
    // 16-bit outputs with unit stride along r: eight consecutive values
    // (16 bytes) per thread on full tiles with aligned rows
    const bool wide = t.out_r == 1 && r0 + TT <= t.rows && c0 + TT <= t.cols && (t.out_c % 8) == 0 &&
                      (reinterpret_cast<uintptr_t>(op + r0) % 16) == 0;
    if (wide) {
      const int g8 = threadIdx.x & 7, cy = threadIdx.x >> 3;  // 8 groups of 8 rows x 32 columns
#pragma unroll
      for (int i = cy; i < TT; i += 32) {
        union {
          TO v[8];
          uint4 u;
        } pk;
#pragma unroll
        for (int q = 0; q < 8; ++q) pk.v[q] = tile[g8 * 8 + q][i];
        *reinterpret_cast<uint4*>(op + (c0 + i) * t.out_c + r0 + g8 * 8) = pk.u;
      }
      return;
    }
  }
  const int px = threadIdx.x & 31, py = threadIdx.x >> 5;  // 32 pairs x 8 rows
  const int64_t r = r0 + 2 * px;
  const bool pair_ok = t.out_r == 1 && r + 1 < t.rows;
#pragma unroll 4
  for (int i = py; i < TT; i += 8) {
    const int64_t c = c0 + i;
    if (c >= t.cols || r >= t.rows) continue;
    TO* p = op + c * t.out_c + r * t.out_r;
    const TO v0 = tile[2 * px][i];
    if (pair_ok && (reinterpret_cast<uintptr_t>(p) % sizeof(Pair<TO>)) == 0) {
      Pair<TO> pr;
      pr.v[0] = v0;
      pr.v[1] = tile[2 * px + 1][i];
      *reinterpret_cast<Pair<TO>*>(p) = pr;
    } else {
      p[0] = v0;
      if (r + 1 < t.rows) p[t.out_r] = tile[2 * px + 1][i];
    }
  }
}
template <typename TI, typename TO>
static hipError_t transpose_t(const void* in, void* out, const TransposeArgs& t, hipStream_t s) {
  const int64_t tr = (t.rows + TT - 1) / TT, tc = (t.cols + TT - 1) / TT;
  const int64_t nz = t.nzb * t.nzc;
  if (tr == 0 || tc == 0 || nz == 0) return hipSuccess;
  hipLaunchKernelGGL((transpose_kernel<TI, TO>), dim3((unsigned)(tr * tc), (unsigned)nz),
                     dim3(256), 0, s, static_cast<const TI*>(in), static_cast<TO*>(out), t, tr, tc);
  return hipGetLastError();
}
hipError_t transpose_cast(int in_dtype, const void* in, int out_dtype, void* out,
                          const TransposeArgs& t, hipStream_t s) {
  ITN_DISPATCH2(in_dtype, out_dtype, transpose_t, in, out, t, s);
}

// ------------------------------------------------------------------ W-stage
// One thread per (output row r, position y): consecutive threads take
// consecutive y of one row (coalesced); grid over ((r, y) chunks, x, z).
// A thread per row rather than per position keeps small bond dimensions
// (Y of a few dozen) from leaving most of the GPU idle.
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void wstage_kernel(const TI* __restrict__ in, TO* __restrict__ out,
                                                      WStageArgs a, const int32_t* __restrict__ row_ptr,
                                                      const int64_t* __restrict__ row_off,
                                                      const int64_t* __restrict__ col_off,
                                                      const double* __restrict__ coef) {
  using A = typename std::conditional<sizeof(TI) == 8, double, float>::type;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t r = t / a.Y, y = t % a.Y;
  const int64_t x = blockIdx.y, z = blockIdx.z;
  if (r >= a.nrows) return;
  const TI* ip = in + x * a.isx + z * a.isz + y * a.isy;
  TO* op = out + x * a.osx + z * a.osz + y * a.osy;
  A acc = 0;
  for (int e = row_ptr[r]; e < row_ptr[r + 1]; ++e) acc += (A)coef[e] * (A)ip[col_off[e]];
  op[row_off[r]] = conv<TO, A>(acc);
}
template <typename TI, typename TO>
static hipError_t wstage_t(const void* in, void* out, const WStageArgs& a, const int32_t* rp,
                           const int64_t* ro, const int64_t* co, const double* cf, hipStream_t s) {
  if (a.X == 0 || a.Y == 0 || a.Z == 0 || a.nrows == 0) return hipSuccess;
  dim3 grid((unsigned)((a.nrows * a.Y + 255) / 256), (unsigned)a.X, (unsigned)a.Z);
  hipLaunchKernelGGL((wstage_kernel<TI, TO>), grid, dim3(256), 0, s, static_cast<const TI*>(in),
                     static_cast<TO*>(out), a, rp, ro, co, cf);
  return hipGetLastError();
}
hipError_t wstage(int in_dtype, const void* in, int out_dtype, void* out, const WStageArgs& a,
                  const int32_t* row_ptr, const int64_t* row_off, const int64_t* col_off,
                  const double* coef, hipStream_t s) {
  if (in_dtype == D_BF16) return hipErrorInvalidValue;
  ITN_DISPATCH2(in_dtype, out_dtype, wstage_t, in, out, a, row_ptr, row_off, col_off, coef, s);
}

// ------------------------------------------------------------------ BLAS-1
constexpr int DOT_THREADS = 256;
constexpr int64_t DOT_CHUNK = 1024;  // elements per block

int64_t dot_blocks(int64_t n) {
  int64_t b = (n + DOT_CHUNK - 1) / DOT_CHUNK;
  return b < 1 ? 1 : b;
}

// partial[j * nb + blockIdx.x] = sum over the block's chunk of V_j * w.
__global__ __launch_bounds__(DOT_THREADS) void multi_dot_partial(const double* __restrict__ V,
                                                                  int64_t ldv, int k,
                                                                  const double* __restrict__ w,
                                                                  int64_t n, double* partial) {
  // up to DG vectors per pass: w is read once per pass and the DG sums are
  // reduced together
  constexpr int DG = 16;
  __shared__ double red[DOT_THREADS / 64][DG];
  const int64_t nb = gridDim.x;
  const int64_t lo = blockIdx.x * DOT_CHUNK;
  int64_t hi = lo + DOT_CHUNK;
  if (hi > n) hi = n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j0 = 0; j0 < k; j0 += DG) {
    double acc[DG];
#pragma unroll
    for (int q = 0; q < DG; ++q) acc[q] = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += DOT_THREADS) {
      const double wi = w[i];
#pragma unroll
      for (int q = 0; q < DG; ++q)
        if (j0 + q < k) acc[q] += V[(int64_t)(j0 + q) * ldv + i] * wi;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
      for (int q = 0; q < DG; ++q) acc[q] += __shfl_down(acc[q], off, 64);
    if (lane == 0)
#pragma unroll
      for (int q = 0; q < DG; ++q) red[wave][q] = acc[q];
    __syncthreads();
    if (threadIdx.x < DG && j0 + (int)threadIdx.x < k) {
      double t = 0.0;
      for (int q = 0; q < DOT_THREADS / 64; ++q) t += red[q][threadIdx.x];
      partial[(int64_t)(j0 + threadIdx.x) * nb + blockIdx.x] = t;
    }
    __syncthreads();
  }
}
// out[j] = sum_b partial[j * nb + b], fixed order.
__global__ void multi_dot_final(const double* __restrict__ partial, int64_t nb, int k,
                                double* out) {
  const int j = blockIdx.x;
  if (j >= k) return;
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += blockDim.x) acc += partial[j * nb + b];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = red[0];
}
hipError_t multi_dot(const double* V, int64_t ldv, int k, const double* w, int64_t n,
                     double* partial, double* out, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  const int64_t nb = dot_blocks(n);
  hipLaunchKernelGGL(multi_dot_partial, dim3((unsigned)nb), dim3(DOT_THREADS), 0, s, V, ldv, k, w,
                     n, partial);
  hipLaunchKernelGGL(multi_dot_final, dim3((unsigned)k), dim3(256), 0, s, partial, nb, k, out);
  return hipGetLastError();
}

struct Coefs {
  double c[64];
};
__global__ void lincomb_kernel(const double* __restrict__ V, int64_t ldv, int k, Coefs c,
                               double beta, double* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double acc = (beta != 0.0) ? beta * y[i] : 0.0;
    for (int j = 0; j < k; ++j) acc += c.c[j] * V[j * ldv + i];
    y[i] = acc;
  }
}
hipError_t lincomb(const double* V, int64_t ldv, int k, const double* c, double beta, double* y,
                   int64_t n, hipStream_t s) {
  if (k > 64 || k < 0) return hipErrorInvalidValue;
  Coefs cc;
  for (int j = 0; j < 64; ++j) cc.c[j] = j < k ? c[j] : 0.0;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(lincomb_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, V, ldv, k, cc,
                     beta, y, n);
  return hipGetLastError();
}

// y += scale * sum_j c[j] * V_j with the coefficients in device memory.
__global__ void lincomb_dev_kernel(const double* __restrict__ V, int64_t ldv, int k,
                                   const double* __restrict__ c, double scale, double* __restrict__ y,
                                   int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int j = 0; j < k; ++j) acc += c[j] * V[(int64_t)j * ldv + i];
    y[i] += scale * acc;
  }
}
hipError_t lincomb_dev(const double* V, int64_t ldv, int k, const double* c, double scale, double* y,
                       int64_t n, hipStream_t s) {
  if (n == 0 || k == 0) return hipSuccess;
  hipLaunchKernelGGL(lincomb_dev_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, V, ldv, k, c,
                     scale, y, n);
  return hipGetLastError();
}

__global__ void scale_kernel(double* x, double a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] *= a;
}
hipError_t scale(double* x, double a, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(scale_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, x, a, n);
  return hipGetLastError();
}

// Diagonal of H_eff (FP64): D[a][c][b] = sum_{m0, m2} L[a][m0][a] Wd[m0][m2][c]
// R[b][m2][b], with Wd[m0][m2][c = s1*d + s2] = sum_m1 W1[m0,m1,s1,s1]
// W2[m1,m2,s2,s2].  A thread per (a, b).
__global__ void heff_diag_kernel(const double* __restrict__ L, const double* __restrict__ R,
                                 const double* __restrict__ Wd, int w, int d2, int64_t cl,
                                 int64_t cr, double* __restrict__ D) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < cl * cr;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = t / cr, b = t % cr;
    for (int c = 0; c < d2; ++c) {
      double acc = 0.0;
      for (int m0 = 0; m0 < w; ++m0) {
        const double l = L[(a * w + m0) * cl + a];
        if (l == 0.0) continue;
        for (int m2 = 0; m2 < w; ++m2) acc += l * Wd[(m0 * w + m2) * d2 + c] * R[(b * w + m2) * cr + b];
      }
      D[(a * d2 + c) * cr + b] = acc;
    }
  }
}
hipError_t heff_diag(const double* L, const double* R, const double* Wd, int w, int d2, int64_t cl,
                     int64_t cr, double* D, hipStream_t s) {
  if (cl * cr == 0) return hipSuccess;
  hipLaunchKernelGGL(heff_diag_kernel, dim3(grid_for(cl * cr, 256, 8192)), dim3(256), 0, s, L, R, Wd,
                     w, d2, cl, cr, D);
  return hipGetLastError();
}

// Diagonal entries of one block-sparse environment, E[x][m][x] for the blocks
// whose two link sectors coincide (their channel sector then carries zero
// charge): out[(g + x) * wz + zb + y] = E_block[(x * dm + y) * dd + x].
__global__ void env_diag_gather_kernel(const double* __restrict__ E, const EnvDiagItem* __restrict__ it,
                                       int nitems, int wz, double* __restrict__ out) {
  for (int k = blockIdx.y; k < nitems; k += gridDim.y) {
    const EnvDiagItem e = it[k];
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < e.dd * e.dm;
         t += (int64_t)gridDim.x * blockDim.x) {
      const int64_t x = t / e.dm, y = t % e.dm;
      out[(e.g + x) * wz + e.zb + y] = E[e.src + (x * e.dm + y) * e.dd + x];
    }
  }
}
hipError_t env_diag_gather(const double* E, const EnvDiagItem* items, int nitems, int wz, double* out,
                           hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  hipLaunchKernelGGL(env_diag_gather_kernel, dim3(4, std::min(nitems, 65535)), dim3(256), 0, s, E, items,
                     nitems, wz, out);
  return hipGetLastError();
}

// Diagonal of the block-sparse two-site H_eff, block by block of psi:
// D[a, s1, s2, b] = sum_{i, j} Ld[a][i] Wd[i][j][s1][s2] Rd[b][j] over the
// zero-charge channels i (wzl of them) and j (wzr); indices global within
// each space.
__global__ void qn_heff_diag_kernel(const double* __restrict__ Ld, const double* __restrict__ Rd,
                                    const double* __restrict__ Wd, int wzl, int wzr, int d1, int d2,
                                    const DiagBlock* __restrict__ blk, int nblk, double* __restrict__ D) {
  for (int k = blockIdx.y; k < nblk; k += gridDim.y) {
    const DiagBlock q = blk[k];
    const int64_t cnt = q.da * q.d1 * q.d2 * q.db;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < cnt;
         t += (int64_t)gridDim.x * blockDim.x) {
      const int64_t z = t % q.db, r = t / q.db;
      const int64_t y2 = r % q.d2, r2 = r / q.d2;
      const int64_t y1 = r2 % q.d1, x = r2 / q.d1;
      const double* la = Ld + (q.ga + x) * wzl;
      const double* rb = Rd + (q.gb + z) * wzr;
      const int64_t c = (q.g1 + y1) * d2 + (q.g2 + y2);
      double acc = 0.0;
      for (int i = 0; i < wzl; ++i) {
        if (la[i] == 0.0) continue;
        double u = 0.0;
        for (int j = 0; j < wzr; ++j) u += Wd[((int64_t)i * wzr + j) * d1 * d2 + c] * rb[j];
        acc += la[i] * u;
      }
      D[q.off + t] = acc;
    }
  }
}
hipError_t qn_heff_diag(const double* Ld, const double* Rd, const double* Wd, int wzl, int wzr, int d1, int d2,
                        const DiagBlock* blocks, int nblk, int64_t chunks, double* D, hipStream_t s) {
  if (nblk == 0) return hipSuccess;
  hipLaunchKernelGGL(qn_heff_diag_kernel, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(chunks, 64)),
                     std::min(nblk, 65535)), dim3(256), 0, s, Ld, Rd, Wd, wzl, wzr, d1, d2, blocks, nblk, D);
  return hipGetLastError();
}

// r[i] /= (D[i] - theta), denominators of magnitude below eps clipped to eps
// (Davidson's diagonal preconditioner).
__global__ void precond_diag_kernel(double* __restrict__ r, const double* __restrict__ D, double theta,
                                    double eps, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double den = D[i] - theta;
    if (fabs(den) < eps) den = den < 0.0 ? -eps : eps;
    r[i] /= den;
  }
}
hipError_t precond_diag(double* r, const double* D, double theta, double eps, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(precond_diag_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, r, D, theta,
                     eps, n);
  return hipGetLastError();
}

// x[i] += eps * u_i with u_i uniform in [-1, 1) from the splitmix64 hash of
// (seed, i) (Steele, Lea and Flood's SplitMix64 finaliser): a reproducible
// perturbation that touches every element.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__global__ void add_noise_kernel(double* __restrict__ x, int64_t n, double eps, uint64_t seed) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t r = splitmix64(seed ^ splitmix64((uint64_t)i));
    const double u = (double)(r >> 11) * (1.0 / 9007199254740992.0);  // [0, 1)
    x[i] += eps * (2.0 * u - 1.0);
  }
}
hipError_t add_noise(double* x, int64_t n, double eps, uint64_t seed, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(add_noise_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, x, n, eps, seed);
  return hipGetLastError();
}

template <typename T> __global__ void fill_kernel(T* x, T v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}
hipError_t fill(void* x, int dtype, double v, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned g = grid_for(n, 256, 8192);
  if (dtype == D_F64)
    hipLaunchKernelGGL(fill_kernel<double>, dim3(g), dim3(256), 0, s, (double*)x, v, n);
  else if (dtype == D_F32)
    hipLaunchKernelGGL(fill_kernel<float>, dim3(g), dim3(256), 0, s, (float*)x, (float)v, n);
  else
    hipLaunchKernelGGL(fill_kernel<bf16_t>, dim3(g), dim3(256), 0, s, (bf16_t*)x,
                       (bf16_t)(float)v, n);
  return hipGetLastError();
}

}  // namespace itn
