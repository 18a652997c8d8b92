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
template <> __device__ __forceinline__ bf16_t qconv<bf16_t>(double x) { return bf16_from_double(x); }

__global__ void qn_set_ptrs_kernel(QnDevPtrs* dst, QnDevPtrs v) {
  if (threadIdx.x == 0) *dst = v;
}
hipError_t qn_set_ptrs(QnDevPtrs* dst, QnDevPtrs v, hipStream_t s) {
  hipLaunchKernelGGL(qn_set_ptrs_kernel, dim3(1), dim3(64), 0, s, dst, v);
  return hipGetLastError();
}

// ------------------------------------------------------------ transpose
// One 64 x 64 tile per workgroup; tile -> block from a table built by the
// planner.  Each element is converted once, as it is loaded, to the output
// type (FP64 -> bf16 is a single rounding, not one to FP32 and another to
// bf16), and the LDS tile holds the converted values.  Output rows are
// padded to a multiple of 8 elements, 16-byte aligned and zero past `rows`,
// so the store phase writes whole 16-byte vectors of consecutive r (zeros
// past `rows`): one store per 8 bf16 instead of one per element.
template <typename TI, typename TO>
__device__ __forceinline__ void transpose_tile(const QnPtrs* __restrict__ ptrs, TO* __restrict__ out,
                                               const QnTBlock* __restrict__ blocks,
                                               const int32_t* __restrict__ tile_block, int t,
                                               int64_t v, int64_t in_bs, int64_t out_bs) {
  __shared__ TO tile[64][65];
  const QnTBlock bk = blocks[tile_block[t]];
  const int local = t - bk.tile0;
  const int64_t r0 = (int64_t)(local / bk.tiles_c) * 64, c0 = (int64_t)(local % bk.tiles_c) * 64;
  const TI* ip = static_cast<const TI*>(ptrs->psi) + bk.in_off + v * in_bs;
  TO* op = out + bk.out_off + v * out_bs;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  // all 16 loads of a thread in flight before the first LDS write
  TI in[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int64_t r = r0 + ty + 4 * k, c = c0 + tx;
    in[k] = r < bk.rows && c < bk.cols ? ip[r * bk.in_ld + c] : TI(0);
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) tile[ty + 4 * k][tx] = qconv<TO>((double)in[k]);
  __syncthreads();
  constexpr int V = 16 / (int)sizeof(TO);  // elements per 16-byte vector
  constexpr int CH = 64 / V;               // vectors per tile column
  union Vec {
    uint4 u;
    TO e[V];
  };
#pragma unroll
  for (int it = threadIdx.x; it < 64 * CH; it += 256) {
    const int ci = it / CH, j = it % CH;
    const int64_t c = c0 + ci, r = r0 + (int64_t)j * V;
    if (c >= bk.cols || r >= bk.rows) continue;
    Vec w;
#pragma unroll
    for (int e = 0; e < V; ++e)
      w.e[e] = r + e < bk.rows ? tile[j * V + e][ci] : qconv<TO>(0.0);
    *reinterpret_cast<uint4*>(op + c * bk.ld_out + r) = w.u;
  }
}

template <typename TI, typename TO>
__global__ __launch_bounds__(256) void qn_transpose_kernel(const QnPtrs* __restrict__ ptrs,
                                                            TO* __restrict__ out,
                                                            const QnTBlock* __restrict__ blocks,
                                                            const int32_t* __restrict__ tile_block,
                                                            int64_t in_bs, int64_t out_bs) {
  transpose_tile<TI, TO>(ptrs, out, blocks, tile_block, blockIdx.x, blockIdx.y, in_bs, out_bs);
}

template <typename TI, typename TO>
static hipError_t qn_transpose_t(const QnPtrs* ptrs, void* out, const QnTBlock* blocks,
                                 const int32_t* tile_block, int64_t ntiles, int64_t in_bs,
                                 int64_t out_bs, int nv, hipStream_t s) {
  if (ntiles == 0 || nv == 0) return hipSuccess;
  hipLaunchKernelGGL((qn_transpose_kernel<TI, TO>), dim3((unsigned)ntiles, (unsigned)nv), dim3(256),
                     0, s, ptrs, static_cast<TO*>(out), blocks, tile_block, in_bs, out_bs);
  return hipGetLastError();
}

hipError_t qn_block_transpose(int in_dtype, const QnPtrs* ptrs, int out_dtype, void* out,
                              const QnTBlock* blocks, const int32_t* tile_block, int64_t ntiles,
                              int64_t in_bs, int64_t out_bs, int nv, hipStream_t s) {
#define ITN_QT(TI, TO) return qn_transpose_t<TI, TO>(ptrs, out, blocks, tile_block, ntiles, in_bs, out_bs, nv, s)
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
// Z[a', s1', s2', m2, b] = sum of coef * X[a', m0, s1, s2, b] over the W12
// terms of the row (s1', s2', m2), for one (a'-sector, b-sector) pair per
// work item.  A work item is one wave: lane l takes vectors v0 + l + 64 k
// (k < NPV), each V consecutive b of one a' (the planner's padding keeps
// every such vector aligned and inside its row), one 16-byte load per entry.
// A workgroup runs four independent items, so a pair of a few dozen vectors
// occupies one wave instead of a whole workgroup.  Entries are taken NE at
// a time, so every lane has NE * NPV independent 16-byte loads in flight
// before it accumulates; Z is written one 16-byte vector per row end, with
// nontemporal stores when `stream` is set (Z larger than the caches).
typedef unsigned int qn_u32x4 __attribute__((ext_vector_type(4)));
template <typename T> union QnVec {
  static constexpr int V = 16 / (int)sizeof(T);
  uint4 u;
  T e[V];
};

template <typename T, int NPV, int NE, bool STREAM>
__global__ __launch_bounds__(256) void qn_wstage_kernel(const T* __restrict__ X, T* __restrict__ Z,
                                                        const QnWPair* __restrict__ pairs,
                                                        const QnWEnt* __restrict__ ents,
                                                        const QnWItem* __restrict__ items,
                                                        int64_t nitems, int64_t x_bs, int64_t z_bs) {
  using A = typename std::conditional<sizeof(T) == 8, double, float>::type;
  constexpr int V = QnVec<T>::V;
  const int lane = threadIdx.x & 63;
  // the item index is uniform over the wave: readfirstlane makes that
  // explicit, so the item, pair and entry records are scalar loads
  const int64_t item = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (item >= nitems) return;  // the whole wave
  const QnWItem it = items[item];
  const QnWPair pr = pairs[it.pair];
  const int vrow = pr.db / V;  // vectors per a'-row
  const int nvec = pr.da * vrow;
  int64_t a[NPV], b[NPV];
  bool ok[NPV];
#pragma unroll
  for (int k = 0; k < NPV; ++k) {
    const int vi = it.v0 + k * 64 + lane;
    ok[k] = vi < nvec;
    const int vv = ok[k] ? vi : 0;  // vector 0 exists in every pair
    a[k] = vv / vrow;
    b[k] = (int64_t)(vv - (int)a[k] * vrow) * V;
  }
  const int64_t v = blockIdx.y;
  const T* xv = X + v * x_bs;
  T* zv = Z + v * z_bs;
  const QnWEnt* en = ents + pr.e0;
  const int ne = pr.ne;
  A z[NPV][V];
#pragma unroll
  for (int k = 0; k < NPV; ++k)
#pragma unroll
    for (int i = 0; i < V; ++i) z[k][i] = 0;
  for (int e0 = 0; e0 < ne; e0 += NE) {
    QnWEnt ec[NE];
    QnVec<T> x[NE][NPV];
#pragma unroll
    for (int j = 0; j < NE; ++j) ec[j] = en[e0 + j < ne ? e0 + j : ne - 1];
#pragma unroll
    for (int j = 0; j < NE; ++j)
#pragma unroll
      for (int k = 0; k < NPV; ++k)
        x[j][k].u = *reinterpret_cast<const uint4*>(xv + ec[j].off + a[k] * ec[j].astride + b[k]);
#pragma unroll
    for (int j = 0; j < NE; ++j) {
      if (e0 + j >= ne) break;
      if (ec[j].coef != 0.0) {  // zero-weight entries of rows without W12 terms add nothing
        const A c = (A)ec[j].coef;
#pragma unroll
        for (int k = 0; k < NPV; ++k)
#pragma unroll
          for (int i = 0; i < V; ++i) z[k][i] += c * (A)x[j][k].e[i];
      }
      if (ec[j].end) {
#pragma unroll
        for (int k = 0; k < NPV; ++k) {
          QnVec<T> o;
#pragma unroll
          for (int i = 0; i < V; ++i) {
            o.e[i] = (T)z[k][i];
            z[k][i] = 0;
          }
          if (ok[k]) {
            T* dst = zv + ec[j].zoff + a[k] * ec[j].zastride + b[k];
            if constexpr (STREAM)
              __builtin_nontemporal_store(__builtin_bit_cast(qn_u32x4, o.u), reinterpret_cast<qn_u32x4*>(dst));
            else
              *reinterpret_cast<uint4*>(dst) = o.u;
          }
        }
      }
    }
  }
}

template <typename T>
static hipError_t qn_wstage_t(const void* X, void* Z, const QnWPair* pairs, const QnWEnt* ents,
                              const QnWItem* items, int64_t nitems, int64_t x_bs, int64_t z_bs,
                              int nv, int per_item, int stream, hipStream_t s) {
  if (nitems == 0 || nv == 0) return hipSuccess;
  const dim3 grid((unsigned)((nitems + 3) / 4), (unsigned)nv);
  const T* x = static_cast<const T*>(X);
  T* z = static_cast<T*>(Z);
#define ITN_QW(NPV, NE)                                                                             \
  do {                                                                                              \
    if (stream)                                                                                     \
      hipLaunchKernelGGL((qn_wstage_kernel<T, NPV, NE, true>), grid, dim3(256), 0, s, x, z, pairs,   \
                         ents, items, nitems, x_bs, z_bs);                                          \
    else                                                                                            \
      hipLaunchKernelGGL((qn_wstage_kernel<T, NPV, NE, false>), grid, dim3(256), 0, s, x, z, pairs,  \
                         ents, items, nitems, x_bs, z_bs);                                          \
  } while (0)
  switch (per_item) {
    case 64: ITN_QW(1, 8); break;
    case 128: ITN_QW(2, 8); break;
    case 256: ITN_QW(4, 4); break;
    default: return hipErrorInvalidValue;
  }
#undef ITN_QW
  return hipGetLastError();
}

hipError_t qn_wstage(int dtype, const void* X, void* Z, const QnWPair* pairs, const QnWEnt* ents,
                     const QnWItem* items, int64_t nitems, int64_t x_bs, int64_t z_bs, int nv,
                     int per_item, int stream, hipStream_t s) {
  if ((x_bs | z_bs) & 7) return hipErrorInvalidValue;  // batch strides keep the 16-byte alignment
  switch (dtype) {
    case D_F64: return qn_wstage_t<double>(X, Z, pairs, ents, items, nitems, x_bs, z_bs, nv, per_item, stream, s);
    case D_F32: return qn_wstage_t<float>(X, Z, pairs, ents, items, nitems, x_bs, z_bs, nv, per_item, stream, s);
    case D_BF16: return qn_wstage_t<bf16_t>(X, Z, pairs, ents, items, nitems, x_bs, z_bs, nv, per_item, stream, s);
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------ block copy
// Rows of an item (at most 32) are spread over the four waves, columns over
// the lanes; narrow blocks use a flat index instead.
template <typename T>
__device__ __forceinline__ void copy_item(const QnPtrs* __restrict__ ptrs, T* __restrict__ outL,
                                          T* __restrict__ outR, const QnCopy& it) {
  const T* src = static_cast<const T*>(it.src ? ptrs->R : ptrs->L) + it.in_off;
  T* dst = (it.src ? outR : outL) + it.out_off;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (it.cols >= 48) {
    for (int r = wave; r < it.rows; r += 4) {
      const T* sr = src + (int64_t)r * it.cols;
      T* dr = dst + (int64_t)r * it.ld_out;
#pragma unroll 4
      for (int c = lane; c < it.cols; c += 64) dr[c] = sr[c];
    }
  } else {
    const int n = it.rows * it.cols;
    const unsigned cols = (unsigned)it.cols;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
      const unsigned r = (unsigned)e / cols, c = (unsigned)e - r * cols;
      dst[(int64_t)r * it.ld_out + c] = src[e];
    }
  }
}
template <typename T>
__global__ __launch_bounds__(256) void qn_copy_kernel(const QnPtrs* __restrict__ ptrs,
                                                       T* __restrict__ outL, T* __restrict__ outR,
                                                       const QnCopy* __restrict__ items) {
  copy_item<T>(ptrs, outL, outR, items[blockIdx.x]);
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

// ------------------------------------------------ repack + transpose
// The L/R repack and the psi transpose of an apply with environments in one
// launch (they are independent): workgroups [0, ncopy) copy one repack item
// each, the rest take the transpose tiles of every vector; one launch
// instead of two dependent ones, and the two passes' tails overlap.
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void qn_prep_kernel(const QnPtrs* __restrict__ ptrs,
                                                       TO* __restrict__ psiT,
                                                       const QnTBlock* __restrict__ blocks,
                                                       const int32_t* __restrict__ tile_block,
                                                       int64_t ntiles, int64_t in_bs, int64_t out_bs,
                                                       TO* __restrict__ outL, TO* __restrict__ outR,
                                                       const QnCopy* __restrict__ items, int64_t ncopy) {
  const int64_t b = blockIdx.x;
  if (b < ncopy) {
    copy_item<TO>(ptrs, outL, outR, items[b]);
    return;
  }
  const int64_t t = (b - ncopy) % ntiles, v = (b - ncopy) / ntiles;
  transpose_tile<TI, TO>(ptrs, psiT, blocks, tile_block, (int)t, v, in_bs, out_bs);
}

template <typename TI, typename TO>
static hipError_t qn_prep_t(const QnPtrs* ptrs, void* psiT, const QnTBlock* blocks,
                            const int32_t* tile_block, int64_t ntiles, int64_t in_bs, int64_t out_bs,
                            int nv, void* outL, void* outR, const QnCopy* items, int64_t ncopy,
                            hipStream_t s) {
  const int64_t n = ncopy + ntiles * nv;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((qn_prep_kernel<TI, TO>), dim3((unsigned)n), dim3(256), 0, s, ptrs,
                     static_cast<TO*>(psiT), blocks, tile_block, ntiles > 0 ? ntiles : 1, in_bs, out_bs,
                     static_cast<TO*>(outL), static_cast<TO*>(outR), items, ncopy);
  return hipGetLastError();
}

hipError_t qn_prepare(int in_dtype, const QnPtrs* ptrs, int out_dtype, void* psiT,
                      const QnTBlock* blocks, const int32_t* tile_block, int64_t ntiles, int64_t in_bs,
                      int64_t out_bs, int nv, void* outL, void* outR, const QnCopy* items,
                      int64_t ncopy, hipStream_t s) {
  if (nv <= 0) ntiles = 0;
#define ITN_QP(TI, TO) \
  return qn_prep_t<TI, TO>(ptrs, psiT, blocks, tile_block, ntiles, in_bs, out_bs, nv, outL, outR, items, ncopy, s)
  if (in_dtype == D_F64) {
    if (out_dtype == D_F64) ITN_QP(double, double);
    if (out_dtype == D_F32) ITN_QP(double, float);
    if (out_dtype == D_BF16) ITN_QP(double, bf16_t);
  } else if (in_dtype == D_F32) {
    if (out_dtype == D_F64) ITN_QP(float, double);
    if (out_dtype == D_F32) ITN_QP(float, float);
    if (out_dtype == D_BF16) ITN_QP(float, bf16_t);
  }
#undef ITN_QP
  return hipErrorInvalidValue;
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
