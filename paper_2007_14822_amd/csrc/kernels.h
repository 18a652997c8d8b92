// Host-side launch interface of the libitn device kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace itn {

// Storage dtypes (same codes as itn_dtype).
enum DType { D_F64 = 0, D_F32 = 1, D_BF16 = 2 };
inline int dtype_size(int dt) { return dt == D_F64 ? 8 : (dt == D_F32 ? 4 : 2); }

// C[b][m][n] = sum_k A[b][m][k] * B[b][n][k]  (both operands K-contiguous,
// "NT").  A, B hold the operand precision's type; C is written as c_dtype.
// If accumulate != 0 the result is added to C (read in c_dtype).
struct GemmArgs {
  const void* A;
  const void* B;
  void* C;
  int64_t M, N, K;
  int64_t lda, ldb, ldc;
  int64_t sA, sB, sC;  // batch strides (elements)
  int32_t batch;
  int32_t accumulate;
  int32_t stream;  // non-zero: C is written with nontemporal stores (read only by a later pass)
};
hipError_t gemm_nt(int prec, int c_dtype, const GemmArgs& g, hipStream_t s);

// Grouped NT GEMM over a device work table: every work item is one output
// tile of one problem; a problem's K is the concatenation of `nseg`
// segments, each with its own A/B base pointers and leading dimensions, and
// is summed in segment order by the single workgroup that owns the tile.
struct GSeg {      // one K segment of one problem
  int64_t a_off;   // element offset of the segment's A block (row 0, k 0)
  int64_t b_off;   // element offset of the segment's B block
  int32_t lda, ldb;
  int32_t K;
  int32_t pad;
};
struct GProb {     // one output problem (an output block, or a group of them)
  int64_t c_off;   // element offset of C (row 0, col 0)
  int32_t M, N;
  int32_t ldc;
  int32_t seg0;    // first segment index
  int32_t nseg;
  int32_t tiles_n; // column tiles
  int32_t row0;    // >= 0: row r of C starts at bases->rows[row0 + r] (c_off, ldc unused)
  int32_t pad;
};
struct GTile {     // one work item
  int32_t prob;    // -1: no work (padding of the tile list)
  int32_t tm, tn;  // tile coordinates within the problem
  int32_t pad;
};
// Base pointers of a grouped launch, read by the kernel from device memory.
struct GBases {
  const void* A;
  const void* B;
  void* C;
  const void* zero;    // >= 16 zero bytes (K tails of direct-to-LDS tiles)
  const int64_t* rows; // row offsets of C for problems with row0 >= 0 (else unused)
  int32_t stream;      // non-zero: C (2-byte) is written with nontemporal stores
  int32_t pad;
};
// Persistent grouped launch: at most max_wg workgroups (0: one per tile)
// stride over the tile list; with max_wg and the list length multiples of
// 8, list position i runs on XCD i % 8.  Tile config: 0 = 64x64, 1 = 128x128 (register
// staged, any alignment); 2 = direct-to-LDS 8-wave tiles (256x256, FP64
// 256x128), 3 = direct-to-LDS 4-wave 128x128 tiles, 4 = direct-to-LDS
// 4-wave 256x64 tiles (narrow products); 2, 3 and 4 need 16-byte aligned
// operand rows that are zero up to K rounded to 16 bytes, and bases->zero.  Batch b (grid.y) offsets A, B and
// C by b times their batch strides.
hipError_t gemm_grouped(int prec, int c_dtype, int tile_cfg, const GBases* bases, const GProb* probs,
                        const GSeg* segs, const GTile* tiles, int64_t ntiles, int64_t a_batch_stride,
                        int64_t b_batch_stride, int64_t c_batch_stride, int nbatch, int max_wg,
                        hipStream_t s);
int grouped_tile_rows(int tile_cfg);
int grouped_tile_cols(int prec, int tile_cfg);

// ------------------------------------------------------------- QN helpers
// Pointers of the caller's operands for one block-sparse H_eff apply, read
// by the kernels from device memory (set by qn_set_ptrs before a replay).
struct QnPtrs {
  const void* L;
  const void* R;
  const void* psi;
  void* out;
};
struct QnDevPtrs {
  QnPtrs p;
  GBases g1;  // stage 1: A = L, B = psiT, C = X
  GBases g4;  // stage 4: A = Z, B = R, C = out
};
hipError_t qn_set_ptrs(QnDevPtrs* dst, QnDevPtrs v, hipStream_t s);
// Per-block transpose with conversion: item i moves block `in` [rows][cols]
// (row stride in_ld, at in_off of psi + v * in_bs) to out_off of `out` +
// v * out_bs as [cols][rows] with row stride ld_out (elements).
struct QnTBlock {
  int64_t in_off, out_off;
  int32_t rows, cols;
  int32_t ld_out;
  int32_t tiles_c;  // column tiles of 64
  int32_t tile0;    // first tile index of this block in the flat tile space
  int32_t in_ld;
};
hipError_t qn_block_transpose(int in_dtype, const QnPtrs* ptrs, int out_dtype, void* out,
                              const QnTBlock* blocks, const int32_t* tile_block, int64_t ntiles,
                              int64_t in_bs, int64_t out_bs, int nv, hipStream_t s);
// Block copy into a padded layout: item i copies rows [0, rows) x [0, cols)
// of a row-major block of the caller's L (src = 0) or R (src = 1) at in_off
// to outL (src = 0) or outR (src = 1) + out_off with row stride ld_out.
struct QnCopy {
  int64_t in_off, out_off;
  int32_t rows, cols;
  int32_t ld_out;
  int32_t src;
};
hipError_t qn_block_copy(int dtype, const QnPtrs* ptrs, void* outL, void* outR,
                         const QnCopy* items, int64_t nitems, hipStream_t s);
// qn_block_copy (ncopy items, in the transpose's output type) and
// qn_block_transpose in one launch (independent passes of an apply).
hipError_t qn_prepare(int in_dtype, const QnPtrs* ptrs, int out_dtype, void* psiT,
                      const QnTBlock* blocks, const int32_t* tile_block, int64_t ntiles, int64_t in_bs,
                      int64_t out_bs, int nv, void* outL, void* outR, const QnCopy* items,
                      int64_t ncopy, hipStream_t s);
// Block-sparse W-stage.  The entries of one (a'-sector, b-sector) pair are
// stored row after row; the last entry of a row carries the row's Z offset,
// and rows without W12 terms have one zero-weight entry, so every Z element
// of the pair is written.  The planner pads every b-sector of X and Z to a
// multiple of 8 columns (db below is the padded width; X padding is zero)
// and keeps every offset and stride a multiple of 8 elements, so the kernel
// moves whole 16-byte vectors of V = 16 / sizeof(T) positions (a', b..b+V-1).
struct QnWPair {
  int32_t e0, ne;       // entries of this pair
  int32_t da, db;       // positions a' < da, b < db (db a multiple of 8)
};
struct QnWEnt {
  int64_t off;          // X offset of (a' = 0, b = 0)
  int64_t astride;
  double coef;
  int64_t zoff;         // Z offset of (a' = 0, b = 0) of the row (last entry of a row)
  int64_t zastride;     // 0 on entries that do not end a row
  int32_t end;          // 1 on the last entry of a row
  int32_t pad;
};
struct QnWItem {
  int32_t pair;
  int32_t v0;  // first vector (position v0 * V in a' * db + b order)
};
// Work items of `per_item` vectors (64, 128 or 256), one wave each (one,
// two or four vectors per lane), four per workgroup; X and Z of batch v at
// v * x_bs, v * z_bs; stream != 0: Z written with nontemporal stores.
// dtype: F64, F32 or BF16 (X and Z alike).
hipError_t qn_wstage(int dtype, const void* X, void* Z, const QnWPair* pairs, const QnWEnt* ents,
                     const QnWItem* items, int64_t nitems, int64_t x_bs, int64_t z_bs, int nv,
                     int per_item, int stream, hipStream_t s);
// Zero the listed output blocks (offsets, sizes) of out + v * bs.
hipError_t qn_zero_blocks(int dtype, const QnPtrs* ptrs, const int64_t* offs, const int64_t* sizes,
                          int nblocks, int64_t bs, int nv, hipStream_t s);

// Generic strided permutation with dtype conversion (rank <= 8):
// out[i_0..i_{r-1}] (row-major over out_dims) = in[sum_k i_k * in_strides[k]].
hipError_t permute_cast(int in_dtype, const void* in, int out_dtype, void* out, int rank,
                        const int64_t* out_dims, const int64_t* in_strides, hipStream_t s);

// Many permutations in one launch (the blocks of a block-sparse operand):
// item i moves out[dst + j] = in[src + sum_k j_k * istr[k]] for the n
// elements j (row-major over dims[0..rank)); the launch runs one workgroup
// per chunk {item, first element} of at most PERM_CHUNK elements.
constexpr int PERM_CHUNK = 4096;
struct PermItem {
  int64_t src, dst, n;
  int32_t rank, pad;
  int64_t dims[8];
  int64_t istr[8];
};
struct PermChunk {
  int32_t item, pad;
  int64_t first;
};
hipError_t permute_batch(int in_dtype, const void* in, int out_dtype, void* out, const PermItem* items,
                         const PermChunk* chunks, int64_t nchunks, hipStream_t s);
// Many strided FP64 2D copies in one launch: item i copies rows x cols
// elements, dst[r * ldd + c] = src[r * lds + c] (lds < 0 walks the source
// rows backwards); one workgroup per chunk {item, first element} of at most
// PERM_CHUNK elements.  Items must not overlap in their destinations.
struct Copy2D {
  const double* src;
  double* dst;
  int64_t rows, cols, lds, ldd;
};
hipError_t copy2d_batch(const Copy2D* items, const PermChunk* chunks, int64_t nchunks, hipStream_t s);

// Batched 2-D transpose with conversion: for each batch z (two levels zb, zc):
//   out[zb][zc][c][r] = in[zb][zc][r][c]  with explicit strides.
struct TransposeArgs {
  int64_t rows, cols;
  int64_t nzb, nzc;
  int64_t in_zb, in_zc, in_r, in_c;     // input strides
  int64_t out_zb, out_zc, out_c, out_r; // output strides
};
hipError_t transpose_cast(int in_dtype, const void* in, int out_dtype, void* out,
                          const TransposeArgs& t, hipStream_t s);

// Sparse "W-stage": for every position (x, z, y)
//   out[x*osx + z*osz + y*osy + row_off[r]] = sum_{e in row r} coef[e] * in[x*isx + z*isz + y*isy + col_off[e]]
// row_ptr has nrows+1 entries.  Inputs are FP64 or FP32 (in_dtype), output
// out_dtype; arithmetic in FP64 for FP64 input, FP32 otherwise.
struct WStageArgs {
  int64_t X, Z, Y;
  int64_t isx, isz, isy;
  int64_t osx, osz, osy;
  int32_t nrows;
};
hipError_t wstage(int in_dtype, const void* in, int out_dtype, void* out, const WStageArgs& a,
                  const int32_t* row_ptr, const int64_t* row_off, const int64_t* col_off,
                  const double* coef, hipStream_t s);

// Fused first stage of H_eff for small w*d^2: X = L psi (MFMA) with the
// W-stage applied in the epilogue, writing Z directly.  See heff.hip.
struct HeffFusedArgs {
  const void* L;     // [chi_l, w, chi_l]
  const void* psiT;  // [d2, nv, chi_r, chi_l]
  void* Z;           // [nv, chi_l, d2, w, chi_r]
  int64_t chi_l, chi_r;
  int32_t w, d2, nv;
  int32_t nrows;     // CSR rows = d2*w (output (c', m2)), at most 63
  int32_t nnz;       // CSR entries, at most 128
  const int32_t* row_ptr;
  const int32_t* col_idx;  // input index m0*d2 + c
  const float* coef32;
  const double* coef64;
};
bool heff_fused_supported(int prec, int w, int d2);
bool heff_fused_table_fits(int nrows, int64_t nnz);
// L and psiT each below 2^31 bytes (the kernel addresses them through buffer
// descriptors); larger problems take the unfused path.
bool heff_fused_fits(int prec, int64_t chi_l, int64_t chi_r, int w, int d2, int nv);
hipError_t heff_stage1_fused(int prec, const HeffFusedArgs& a, hipStream_t s);

// Element-wise conversion of a contiguous buffer.
hipError_t cast(int in_dtype, const void* in, int out_dtype, void* out, int64_t n, hipStream_t s);

// FP64 BLAS-1 helpers for the eigensolver (deterministic reductions).
// out[j] = <V_j, w> for k vectors V_j = V + j*ldv, length n.  `partial`
// must hold k * dot_blocks(n) doubles.
int64_t dot_blocks(int64_t n);
hipError_t multi_dot(const double* V, int64_t ldv, int k, const double* w, int64_t n,
                     double* partial, double* out, hipStream_t s);
// y = sum_j c[j] * V_j  (+ beta*y if beta != 0); c on host, k <= 64.
hipError_t lincomb(const double* V, int64_t ldv, int k, const double* c, double beta, double* y,
                   int64_t n, hipStream_t s);
hipError_t scale(double* x, double a, int64_t n, hipStream_t s);
// y += scale * sum_j c[j] * V_j, coefficients c (k of them) in device memory.
hipError_t lincomb_dev(const double* V, int64_t ldv, int k, const double* c, double scale, double* y,
                       int64_t n, hipStream_t s);
hipError_t fill(void* x, int dtype, double v, int64_t n, hipStream_t s);
// Diagonal of the dense H_eff (FP64): L [cl, w, cl], R [cr, w, cr], Wd [w][w][d2]
// (Wd[m0][m2][s1*d + s2] = sum_m1 W1[m0,m1,s1,s1] W2[m1,m2,s2,s2]), D [cl, d2, cr].
hipError_t heff_diag(const double* L, const double* R, const double* Wd, int w, int d2, int64_t cl,
                     int64_t cr, double* D, hipStream_t s);
// Block-sparse H_eff diagonal.  EnvDiagItem: one environment block whose two
// link sectors coincide, data at `src` as [dd][dm][dd]; its diagonal goes to
// out[(g + x) * wz + zb + y] (g: the link sector's global offset, zb: the
// channel sector's first position among the wz zero-charge channels).
struct EnvDiagItem {
  int64_t src, dd, dm, g, zb;
};
hipError_t env_diag_gather(const double* E, const EnvDiagItem* items, int nitems, int wz, double* out,
                           hipStream_t s);
// DiagBlock: one psi block at element offset `off`, extents [da][d1][d2][db],
// global offsets of its sectors ga, g1, g2, gb.  D = sum_{i,j} Ld[a][i]
// Wd[i][j][s1][s2] Rd[b][j] (Ld [chi_l][wzl], Rd [chi_r][wzr],
// Wd [wzl][wzr][d1][d2]).
struct DiagBlock {
  int64_t off, da, d1, d2, db, ga, g1, g2, gb;
};
hipError_t qn_heff_diag(const double* Ld, const double* Rd, const double* Wd, int wzl, int wzr, int d1, int d2,
                        const DiagBlock* blocks, int nblk, int64_t chunks, double* D, hipStream_t s);
// x[i] += eps * (uniform in [-1, 1) from a counter-based hash of (seed, i)).
hipError_t add_noise(double* x, int64_t n, double eps, uint64_t seed, hipStream_t s);
// r /= (D - theta) element-wise, denominators clipped to magnitude >= eps.
hipError_t precond_diag(double* r, const double* D, double theta, double eps, int64_t n, hipStream_t s);

// Householder tridiagonalisation of a symmetric FP64 n x n matrix A (rows of
// length n at stride lda; read only) in one cooperative launch of nwg
// workgroups: d[n], e[n-1] (T[k+1][k] = e[k]), tau[n-1], reflector k in row k
// of V [n][n] (V[k][j] = 0 for j <= k, V[k][k+1] = 1).  Scratch: pub[2n],
// pbuf[2n], dots[2 nwg], bar, err (zeroed by the call).  *err becomes non-zero
// if a grid barrier waited more than spin_limit polls (results invalid).
struct SytrdArgs {
  const double* A;
  int64_t lda;
  int n, nwg, rows_per;
  double *d, *e, *tau, *V, *pub, *pbuf, *dots;
  unsigned* bar;
  int* err;
  int64_t spin_limit;
};
int sytrd_coop_groups(int n);  // workgroup count whose LDS holds A (0: n unsupported)
size_t sytrd_coop_lds(int n, int nwg);
hipError_t sytrd_coop(const SytrdArgs& a, hipStream_t s);
// out[r][:] = Q ZT[:, cols0 - r] for r < k, Q = H_0 H_1 ... H_{n-3} from sytrd_coop.
hipError_t tridiag_back(const double* V, const double* tau, const double* ZT, int64_t ldz, int cols0,
                        double* out, int n, int k, hipStream_t s);
bool tridiag_back_supported(int n);
// Batch of nbatch symmetric nmax x nmax matrices A (column-major, stride
// nmax^2) from per-matrix n x n blocks of rho (meta[2b] = n, meta[2b + 1] =
// offset in rho): rho_b leading, -1 on the rest of the diagonal, 0 elsewhere.
hipError_t pad_batch(const double* rho, const int64_t* meta, double* A, int64_t nmax, int nbatch,
                     hipStream_t s);

}  // namespace itn
