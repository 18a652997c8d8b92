// Memory-bound kernels of the block-sparse (QN) H_eff: per-block transpose
// of psi into the stage-1 operand, the block-sparse W-stage, zero fill of
// output blocks without contributions, and the operand-pointer update used
// before a graph replay.
#include "common.h"
#include "kernels.h"

namespace itn {

template <typename To> __device__ __forceinline__ To qconv(double x) { return (To)(float)x; }
template <> __device__ __forceinline__ double qconv<double>(double x) { return x; }
template <> __device__ __forceinline__ float qconv<float>(double x) { return (float)x; }

__global__ void qn_set_ptrs_kernel(QnDevPtrs* dst, QnDevPtrs v) {
  if (threadIdx.x == 0) *dst = v;
}
hipError_t qn_set_ptrs(QnDevPtrs* dst, QnDevPtrs v, hipStream_t s) {
  hipLaunchKernelGGL(qn_set_ptrs_kernel, dim3(1), dim3(64), 0, s, dst, v);
  return hipGetLastError();
}

// ------------------------------------------------------------ transpose
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void qn_transpose_kernel(const QnPtrs* __restrict__ ptrs,
                                                            TO* __restrict__ out,
                                                            const QnTBlock* __restrict__ blocks,
                                                            int nblocks, int64_t in_bs,
                                                            int64_t out_bs) {
  __shared__ double tile[64][65];
  // locate the block owning this tile (blocks sorted by tile0)
  const int t = blockIdx.x;
  int lo = 0, hi = nblocks - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (blocks[mid].tile0 <= t) lo = mid;
    else hi = mid - 1;
  }
  const QnTBlock bk = blocks[lo];
  const int local = t - bk.tile0;
  const int64_t r0 = (int64_t)(local / bk.tiles_c) * 64, c0 = (int64_t)(local % bk.tiles_c) * 64;
  const int64_t v = blockIdx.y;
  const TI* ip = static_cast<const TI*>(ptrs->psi) + bk.in_off + v * in_bs;
  TO* op = out + bk.out_off + v * out_bs;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < 64; i += 4) {
    const int64_t r = r0 + i, c = c0 + tx;
    if (r < bk.rows && c < bk.cols) tile[i][tx] = (double)ip[r * bk.cols + c];
  }
  __syncthreads();
  for (int i = ty; i < 64; i += 4) {
    const int64_t c = c0 + i, r = r0 + tx;
    if (r < bk.rows && c < bk.cols) op[c * bk.ld_out + r] = qconv<TO>(tile[tx][i]);
  }
}

template <typename TI, typename TO>
static hipError_t qn_transpose_t(const QnPtrs* ptrs, void* out, const QnTBlock* blocks, int nblocks,
                                 int64_t ntiles, int64_t in_bs, int64_t out_bs, int nv,
                                 hipStream_t s) {
  if (ntiles == 0 || nv == 0) return hipSuccess;
  hipLaunchKernelGGL((qn_transpose_kernel<TI, TO>), dim3((unsigned)ntiles, (unsigned)nv), dim3(256),
                     0, s, ptrs, static_cast<TO*>(out), blocks, nblocks, in_bs, out_bs);
  return hipGetLastError();
}

hipError_t qn_block_transpose(int in_dtype, const QnPtrs* ptrs, int out_dtype, void* out,
                              const QnTBlock* blocks, int nblocks, int64_t ntiles, int64_t in_bs,
                              int64_t out_bs, int nv, hipStream_t s) {
#define ITN_QT(TI, TO) return qn_transpose_t<TI, TO>(ptrs, out, blocks, nblocks, ntiles, in_bs, out_bs, nv, s)
  if (in_dtype == D_F64) {
    if (out_dtype == D_F64) ITN_QT(double, double);
    if (out_dtype == D_F32) ITN_QT(double, float);
    if (out_dtype == D_BF16) ITN_QT(double, bf16_t);
  } else if (in_dtype == D_F32) {
    if (out_dtype == D_F64) ITN_QT(float, double);
    if (out_dtype == D_F32) ITN_QT(float, float);
    if (out_dtype == D_BF16) ITN_QT(float, bf16_t);
  }
#undef ITN_QT
  return hipErrorInvalidValue;
}

// -------------------------------------------------------------- W-stage
template <typename TX, typename TZ>
__global__ __launch_bounds__(256) void qn_wstage_kernel(const TX* __restrict__ X, TZ* __restrict__ Z,
                                                         const QnWPair* __restrict__ pairs,
                                                         const QnWRow* __restrict__ rows,
                                                         const QnWEnt* __restrict__ ents,
                                                         const QnWItem* __restrict__ items,
                                                         int64_t x_bs, int64_t z_bs) {
  using A = typename std::conditional<sizeof(TX) == 8, double, float>::type;
  const QnWItem it = items[blockIdx.x];
  const QnWPair pr = pairs[it.pair];
  const int64_t p = (int64_t)it.p0 + threadIdx.x;
  if (p >= (int64_t)pr.da * pr.db) return;
  const int64_t a = p / pr.db, b = p % pr.db;
  const int64_t v = blockIdx.y;
  const TX* xp = X + v * x_bs + b;
  TZ* zp = Z + v * z_bs + b;
  for (int r = pr.row0; r < pr.row0 + pr.nrows; ++r) {
    const QnWRow row = rows[r];
    A z = 0;
    for (int e = row.e0; e < row.e0 + row.ne; ++e) {
      const QnWEnt en = ents[e];
      z += (A)en.coef * (A)xp[en.off + a * en.astride];
    }
    zp[row.off + a * row.astride] = qconv<TZ>((double)z);
  }
}

template <typename TX, typename TZ>
static hipError_t qn_wstage_t(const void* X, void* Z, const QnWPair* pairs, const QnWRow* rows,
                              const QnWEnt* ents, const QnWItem* items, int64_t nitems, int64_t x_bs,
                              int64_t z_bs, int nv, hipStream_t s) {
  if (nitems == 0 || nv == 0) return hipSuccess;
  hipLaunchKernelGGL((qn_wstage_kernel<TX, TZ>), dim3((unsigned)nitems, (unsigned)nv), dim3(256), 0,
                     s, static_cast<const TX*>(X), static_cast<TZ*>(Z), pairs, rows, ents, items,
                     x_bs, z_bs);
  return hipGetLastError();
}

hipError_t qn_wstage(int x_dtype, const void* X, int z_dtype, void* Z, const QnWPair* pairs,
                     const QnWRow* rows, const QnWEnt* ents, const QnWItem* items, int64_t nitems,
                     int64_t x_bs, int64_t z_bs, int nv, hipStream_t s) {
#define ITN_QW(TX, TZ) return qn_wstage_t<TX, TZ>(X, Z, pairs, rows, ents, items, nitems, x_bs, z_bs, nv, s)
  if (x_dtype == D_F64 && z_dtype == D_F64) ITN_QW(double, double);
  if (x_dtype == D_F32 && z_dtype == D_F32) ITN_QW(float, float);
  if (x_dtype == D_F32 && z_dtype == D_BF16) ITN_QW(float, bf16_t);
#undef ITN_QW
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------ block copy
template <typename T>
__global__ __launch_bounds__(256) void qn_copy_kernel(const QnPtrs* __restrict__ ptrs,
                                                       T* __restrict__ outL, T* __restrict__ outR,
                                                       const QnCopy* __restrict__ items) {
  const QnCopy it = items[blockIdx.x];
  const T* src = static_cast<const T*>(it.src ? ptrs->R : ptrs->L) + it.in_off;
  T* dst = (it.src ? outR : outL) + it.out_off;
  // an item holds at most 32 rows: 32-bit index arithmetic
  const int n = it.rows * it.cols;
  const unsigned cols = (unsigned)it.cols;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const unsigned r = (unsigned)e / cols, c = (unsigned)e - r * cols;
    dst[(int64_t)r * it.ld_out + c] = src[e];
  }
}
hipError_t qn_block_copy(int dtype, const QnPtrs* ptrs, void* outL, void* outR,
                         const QnCopy* items, int64_t nitems, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  if (dtype == D_F64)
    hipLaunchKernelGGL(qn_copy_kernel<double>, dim3((unsigned)nitems), dim3(256), 0, s, ptrs,
                       static_cast<double*>(outL), static_cast<double*>(outR), items);
  else if (dtype == D_F32)
    hipLaunchKernelGGL(qn_copy_kernel<float>, dim3((unsigned)nitems), dim3(256), 0, s, ptrs,
                       static_cast<float*>(outL), static_cast<float*>(outR), items);
  else
    hipLaunchKernelGGL(qn_copy_kernel<bf16_t>, dim3((unsigned)nitems), dim3(256), 0, s, ptrs,
                       static_cast<bf16_t*>(outL), static_cast<bf16_t*>(outR), items);
  return hipGetLastError();
}

// ----------------------------------------------------------- zero blocks
template <typename T>
__global__ void qn_zero_kernel(const QnPtrs* __restrict__ ptrs, const int64_t* __restrict__ offs,
                               const int64_t* __restrict__ sizes, int64_t bs) {
  T* o = static_cast<T*>(ptrs->out) + offs[blockIdx.x] + (int64_t)blockIdx.y * bs;
  const int64_t n = sizes[blockIdx.x];
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) o[i] = (T)0;
}
hipError_t qn_zero_blocks(int dtype, const QnPtrs* ptrs, const int64_t* offs, const int64_t* sizes,
                          int nblocks, int64_t bs, int nv, hipStream_t s) {
  if (nblocks == 0 || nv == 0) return hipSuccess;
  if (dtype == D_F64)
    hipLaunchKernelGGL(qn_zero_kernel<double>, dim3(nblocks, nv), dim3(256), 0, s, ptrs, offs, sizes, bs);
  else if (dtype == D_F32)
    hipLaunchKernelGGL(qn_zero_kernel<float>, dim3(nblocks, nv), dim3(256), 0, s, ptrs, offs, sizes, bs);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace itn
