// Symmetric eigensolver pieces for the FP64 bond split: Householder
// tridiagonalisation in one cooperative launch, and the back-transformation
// of selected tridiagonal eigenvectors.
//
// Tridiagonalisation Q^T A Q = T (Householder, one column per step): at step
// k the reflector H_k = I - tau_k v_k v_k^T with v_k[j] = 0 for j <= k and
// v_k[k+1] = 1 annihilates A[k+2:, k]; the trailing block is updated by the
// symmetric rank-2 form A <- A - v w^T - w v^T with p = tau A v,
// w = p - (tau/2)(p^T v) v.  The rows of A are spread cyclically over the
// workgroups of one cooperative launch and stay in LDS for the whole
// reduction; per step only row k+1 (the next pivot row) and p travel between
// workgroups, through global memory and one grid barrier.  One launch
// replaces the per-column launches of a library reduction, whose cost at
// n of a few hundred is launch latency.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace itn {

namespace {

constexpr int EIG_THREADS = 256;

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Sum over the workgroup; every thread gets the result.  `red` holds one
// double per wave.
__device__ __forceinline__ double block_sum(double x, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  x = wave_sum(x);
  __syncthreads();
  if (lane == 0) red[wave] = x;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < EIG_THREADS / 64; ++w) s += red[w];
  return s;
}

// Data exchanged between workgroups inside the launch goes through
// agent-scope atomic stores and loads: coherent across XCDs without
// whole-cache write-back / invalidate fences (which cost several
// microseconds per barrier).
__device__ __forceinline__ void shared_store(double* p, double x) {
  __hip_atomic_store(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double shared_load(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier over the cooperative launch.  Every wave first waits for
// its own stores to complete (so the shared_store data of the step are
// performed before the arrival is counted); arrivals are counted on `bar`
// with agent-scope atomics; the loads after the barrier are issued only
// once the count is seen.  A wait that exceeds `spin_limit` polls sets
// *err and gives up, so every wave always reaches the end of the kernel.
__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned target, int* err,
                                             int64_t spin_limit) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int64_t spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++spins > spin_limit ||
          __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(EIG_THREADS) void sytrd_coop_kernel(SytrdArgs a) {
  extern __shared__ __align__(16) double lds_d[];
  const int n = a.n, nwg = a.nwg, g = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int nrows = (n - g + nwg - 1) / nwg;  // rows g, g + nwg, ... (at most 64)
  const int ld = n | 1;                        // odd row stride: a lane per row hits distinct banks
  double* rows = lds_d;                        // [nrows][ld]
  double* v = rows + (int64_t)a.rows_per * ld; // [n]
  double* w = v + n;                           // [n]
  double* x = w + n;                           // [n] current row k (the pivot row)
  double* part4 = x + n;                       // [EIG_THREADS] per-wave partial row sums
  double* red = part4 + EIG_THREADS;           // [EIG_THREADS / 64 + nwg]
  for (int64_t t = tid; t < (int64_t)nrows * n; t += EIG_THREADS) {
    const int r = (int)(t / n), j = (int)(t % n);
    rows[(int64_t)r * ld + j] = a.A[(int64_t)(g + r * nwg) * a.lda + j];
  }
  for (int j = tid; j < n; j += EIG_THREADS) x[j] = a.A[j];  // row 0
  __syncthreads();
  // One grid barrier per step.  Every workgroup holds the pivot row k: it
  // forms v_k itself, and after the barrier rebuilds row k+1 from the
  // published pre-update copy and this step's rank-2 term.  Published data
  // alternate between two buffers by step parity, so a workgroup that is
  // one step ahead never overwrites what a slower one still reads.
  unsigned epoch = 0;
  for (int k = 0; k + 2 < n; ++k) {
    const int par = k & 1;
    double* pub = a.pub + par * n;
    double* pbuf = a.pbuf + par * n;
    double* dots = a.dots + par * nwg;
    const double alpha = x[k + 1];
    double ss = 0.0;
    for (int j = k + 2 + tid; j < n; j += EIG_THREADS) ss += x[j] * x[j];
    const double xnorm2 = block_sum(ss, red);
    double tau = 0.0, beta = alpha;
    if (xnorm2 > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
      tau = (beta - alpha) / beta;
      const double scal = 1.0 / (alpha - beta);
      for (int j = k + 2 + tid; j < n; j += EIG_THREADS) v[j] = x[j] * scal;
    } else {
      for (int j = k + 2 + tid; j < n; j += EIG_THREADS) v[j] = 0.0;
    }
    if (tid == 0) v[k + 1] = 1.0;
    __syncthreads();
    if (g == 0) {
      if (tid == 0) {
        a.d[k] = x[k];
        a.e[k] = beta;
        a.tau[k] = tau;
      }
      double* vk = a.V + (int64_t)k * n;
      for (int j = tid; j < n; j += EIG_THREADS) vk[j] = j > k ? v[j] : 0.0;
    }
    // row k+1 before this step's update, for every workgroup's next pivot
    if ((k + 1) % nwg == g) {
      const double* rk = rows + (int64_t)((k + 1) / nwg) * ld;
      for (int j = k + 1 + tid; j < n; j += EIG_THREADS) shared_store(pub + j, rk[j]);
    }
    // p = tau A v on this workgroup's rows i > k: lane r sums row r over a
    // quarter of the columns (one quarter per wave); wave 0 adds the four
    // quarters and forms this workgroup's part of p.v
    {
      const int cnt = n - (k + 1), q4 = (cnt + 3) / 4;
      const int j0 = k + 1 + wave * q4, j1 = min(n, j0 + q4);
      double sacc = 0.0;
      if (lane < nrows) {  // four independent sums keep several LDS reads in flight
        const double* ri = rows + (int64_t)lane * ld;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int j = j0;
#pragma unroll 2
        for (; j + 3 < j1; j += 4) {
          s0 += ri[j] * v[j];
          s1 += ri[j + 1] * v[j + 1];
          s2 += ri[j + 2] * v[j + 2];
          s3 += ri[j + 3] * v[j + 3];
        }
        for (; j < j1; ++j) s0 += ri[j] * v[j];
        sacc = (s0 + s1) + (s2 + s3);
      }
      part4[tid] = sacc;
    }
    __syncthreads();
    if (wave == 0) {
      double part = 0.0;
      const int i = g + lane * nwg;
      if (lane < nrows && i > k) {
        const double pi = tau * (((part4[lane] + part4[64 + lane]) + part4[128 + lane]) + part4[192 + lane]);
        shared_store(pbuf + i, pi);
        part = pi * v[i];
      }
      part = wave_sum(part);
      if (lane == 0) shared_store(dots + g, part);
    }
    grid_barrier(a.bar, (++epoch) * (unsigned)nwg, a.err, a.spin_limit);
    // everything published this step, fetched in one batch
    constexpr int MJ = 8;  // n <= 1 + 8 * EIG_THREADS
    double pb[MJ], pu[MJ];
#pragma unroll
    for (int m = 0; m < MJ; ++m) {
      const int j = k + 1 + tid + m * EIG_THREADS;
      pb[m] = j < n && tau != 0.0 ? shared_load(pbuf + j) : 0.0;
      pu[m] = j < n ? shared_load(pub + j) : 0.0;
    }
    if (tid < nwg) red[EIG_THREADS / 64 + tid] = tau != 0.0 ? shared_load(dots + tid) : 0.0;
    __syncthreads();
    double pv = 0.0;
    for (int q = 0; q < nwg; ++q) pv += red[EIG_THREADS / 64 + q];  // fixed order: same in every workgroup
    const double K = -0.5 * tau * pv;
#pragma unroll
    for (int m = 0; m < MJ; ++m) {
      const int j = k + 1 + tid + m * EIG_THREADS;
      if (j < n) w[j] = pb[m] + K * v[j];
    }
    __syncthreads();
    // next pivot row: row k+1 after this step's update
    {
      const double vi = v[k + 1], wi = w[k + 1];
#pragma unroll
      for (int m = 0; m < MJ; ++m) {
        const int j = k + 1 + tid + m * EIG_THREADS;
        if (j < n) x[j] = pu[m] - (vi * w[j] + wi * v[j]);
      }
    }
    if (tau != 0.0) {
      // A_ij -= v_i w_j + w_i v_j on this workgroup's rows i > k, columns j > k
      const int r0 = g > k ? 0 : (k - g) / nwg + 1;  // first row with i > k
#pragma unroll
      for (int m = 0; m < MJ; ++m) {
        const int j = k + 1 + tid + m * EIG_THREADS;
        if (j >= n) break;
        const double vj = v[j], wj = w[j];
#pragma unroll 4
        for (int r = r0; r < nrows; ++r) {
          const int i = g + r * nwg;
          rows[(int64_t)r * ld + j] -= v[i] * wj + w[i] * vj;
        }
      }
    }
    __syncthreads();
  }
  // the last 2x2 block
  const int i0 = n - 2, i1 = n - 1;
  if (i0 % nwg == g && tid == 0) a.d[i0] = rows[(int64_t)(i0 / nwg) * ld + i0];
  if (i1 % nwg == g && tid == 0) {
    a.d[i1] = rows[(int64_t)(i1 / nwg) * ld + i1];
    a.e[i0] = rows[(int64_t)(i1 / nwg) * ld + i0];
    a.tau[i0] = 0.0;
  }
}

// out[r][:] = Q z with z = column cols0 - r of ZT (descending order when
// cols0 = n - 1): reflectors applied last to first.  A workgroup holds VPW
// vectors in LDS (256 / VPW lanes per vector) and streams the reflectors
// through LDS in chunks of C rows of V, loading the next chunk into
// registers while it applies the current one.
template <int VPW, int C>
__global__ __launch_bounds__(256) void tridiag_back_kernel(const double* __restrict__ V,
                                                           const double* __restrict__ tau,
                                                           const double* __restrict__ ZT, int64_t ldz,
                                                           int cols0, double* __restrict__ out, int n,
                                                           int k) {
  constexpr int L = 256 / VPW;  // lanes per vector
  constexpr int PF = 24;        // prefetch registers per thread (C * n <= 256 * PF)
  extern __shared__ __align__(16) double sh[];
  double* z = sh;                          // [VPW][n]
  double* vb = z + (int64_t)VPW * n;       // [2][C][n]
  double* tb = vb + (int64_t)2 * C * n;    // [2][C]
  const int tid = threadIdx.x, grp = tid / L, t = tid % L;
  const int r = blockIdx.x * VPW + grp;
  double* zr = z + (int64_t)grp * n;
  if (r < k) {
    const double* src = ZT + (int64_t)(cols0 - r) * ldz;
    for (int j = t; j < n; j += L) zr[j] = src[j];
  }
  const int nref = n - 2;  // reflectors 0 .. n-3
  const int nchunk = (nref + C - 1) / C;
  // chunk c holds reflectors q = nref-1-c*C-u for u < C (descending)
  double pf[PF];
  double pt = 0.0;
  auto fetch = [&](int c) {
#pragma unroll
    for (int m = 0; m < PF; ++m) {
      const int e = tid + m * 256;
      const int u = e / n, j = e % n;
      const int q = nref - 1 - c * C - u;
      pf[m] = (u < C && q >= 0) ? V[(int64_t)q * n + j] : 0.0;
    }
    const int q = nref - 1 - c * C - tid;
    pt = (tid < C && q >= 0) ? tau[q] : 0.0;
  };
  auto stash = [&](int buf) {
    double* dst = vb + (int64_t)buf * C * n;
#pragma unroll
    for (int m = 0; m < PF; ++m) {
      const int e = tid + m * 256;
      if (e < C * n) dst[e] = pf[m];
    }
    if (tid < C) tb[buf * C + tid] = pt;
  };
  if (nchunk > 0) {
    fetch(0);
    stash(0);
  }
  __syncthreads();
  for (int c = 0; c < nchunk; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunk) fetch(c + 1);
    const double* vc = vb + (int64_t)buf * C * n;
    if (r < k) {
      for (int u = 0; u < C; ++u) {
        const double tq = tb[buf * C + u];
        if (tq == 0.0) continue;  // also the padding past reflector 0
        const double* vq = vc + (int64_t)u * n;
        double sacc = 0.0;
        for (int j = t; j < n; j += L) sacc += vq[j] * zr[j];
#pragma unroll
        for (int off = L / 2; off > 0; off >>= 1) sacc += __shfl_xor(sacc, off, 64);
        sacc *= tq;
        for (int j = t; j < n; j += L) zr[j] -= sacc * vq[j];
      }
    }
    __syncthreads();
    if (c + 1 < nchunk) stash(buf ^ 1);
    __syncthreads();
  }
  if (r < k) {
    double* dst = out + (int64_t)r * n;
    for (int j = t; j < n; j += L) dst[j] = zr[j];
  }
}

// Vectors per workgroup and reflector chunk for n (0: n too large).
static void back_cfg(int n, int& vpw, int& c) {
  vpw = 0;
  c = 0;
  const int cands[3][2] = {{4, 16}, {4, 8}, {4, 4}};  // a wave per vector: k / 4 workgroups
  for (auto& cd : cands) {
    const int64_t lds = ((int64_t)cd[0] * n + 2LL * cd[1] * n + 2 * cd[1]) * 8;
    if (lds <= 160 * 1024 && (int64_t)cd[1] * n <= 256 * 24) {
      vpw = cd[0];
      c = cd[1];
      return;
    }
  }
}

__global__ void zero_u32_kernel(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

}  // namespace

// Per-sector density matrices padded into one batch of nmax x nmax matrices
// (meta[2b] = n, meta[2b + 1] = element offset of sector b's n x n matrix in
// rho): rho_b in the leading block, -1 on the rest of the diagonal, 0
// elsewhere.  The padding is a separate diagonal block whose eigenvalues
// (-1) lie below every density-matrix weight, so the eigenpairs of rho_b are
// those of the padded matrix with the padding rows zero.
__global__ void pad_batch_kernel(const double* __restrict__ rho, const int64_t* __restrict__ meta,
                                 double* __restrict__ A, int64_t nmax) {
  const int64_t b = blockIdx.y;
  const int64_t n = meta[2 * b], off = meta[2 * b + 1];
  double* Ab = A + b * nmax * nmax;
  const int64_t tot = nmax * nmax;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = idx / nmax, r = idx - c * nmax;
    Ab[idx] = (r < n && c < n) ? rho[off + r * n + c] : (r == c ? -1.0 : 0.0);
  }
}

int sytrd_coop_groups(int n) {
  if (n < 3 || n > 1 + 8 * EIG_THREADS) return 0;
  // rows of A plus three n-vectors must fit the LDS of one workgroup
  // (a lane per row in the row sums: at most 64 rows per workgroup)
  // 16 workgroups from n = 192 on (measured at n = 288: 1.62 ms against 1.71
  // with 8 and 1.73 with 32); more only when the rows do not fit
  for (int nwg = n >= 192 ? 16 : 8; nwg <= 256; nwg *= 2) {
    const int64_t rows = (n + nwg - 1) / nwg;
    if (rows <= 64 && sytrd_coop_lds(n, nwg) <= 160 * 1024) return nwg;
  }
  return 0;
}

size_t sytrd_coop_lds(int n, int nwg) {
  const int64_t rows = (n + nwg - 1) / nwg;
  return (size_t)((rows * (n + 1) + 3 * (int64_t)n + EIG_THREADS + EIG_THREADS / 64 + nwg) * 8);
}

hipError_t sytrd_coop(const SytrdArgs& a0, hipStream_t s) {
  SytrdArgs a = a0;
  if (a.n < 3 || a.n > 1 + 8 * EIG_THREADS || a.nwg < 1) return hipErrorInvalidValue;
  a.rows_per = (a.n + a.nwg - 1) / a.nwg;
  if (a.rows_per > 64) return hipErrorInvalidValue;
  const size_t lds = sytrd_coop_lds(a.n, a.nwg);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  static const hipError_t attr = hipFuncSetAttribute(
      reinterpret_cast<const void*>(sytrd_coop_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
      160 * 1024);
  if (attr != hipSuccess) return attr;
  // barrier counter and error flag start at zero (a kernel, not a memset)
  hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, s, a.bar, 1);
  hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned*>(a.err), 1);
  void* args[] = {&a};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(sytrd_coop_kernel), dim3(a.nwg),
                                    dim3(EIG_THREADS), args, (unsigned)lds, s);
}

hipError_t pad_batch(const double* rho, const int64_t* meta, double* A, int64_t nmax, int nbatch,
                     hipStream_t s) {
  if (nmax <= 0 || nbatch <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((nmax * nmax + 255) / 256, 1024);
  hipLaunchKernelGGL(pad_batch_kernel, dim3((unsigned)blocks, (unsigned)nbatch), dim3(256), 0, s, rho,
                     meta, A, nmax);
  return hipGetLastError();
}

bool tridiag_back_supported(int n) {
  int vpw, c;
  back_cfg(n, vpw, c);
  return n >= 3 && vpw > 0;
}

hipError_t tridiag_back(const double* V, const double* tau, const double* ZT, int64_t ldz, int cols0,
                        double* out, int n, int k, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  if (n < 3 || cols0 - (k - 1) < 0 || cols0 >= n) return hipErrorInvalidValue;
  int vpw, c;
  back_cfg(n, vpw, c);
  if (vpw == 0) return hipErrorInvalidValue;
  const size_t lds = ((size_t)vpw * n + 2 * (size_t)c * n + 2 * c) * 8;
  auto go = [&](auto kern) -> hipError_t {
    static const hipError_t attr = hipFuncSetAttribute(
        reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(kern, dim3((unsigned)((k + vpw - 1) / vpw)), dim3(256), lds, s, V, tau, ZT, ldz,
                       cols0, out, n, k);
    return hipGetLastError();
  };
  if (c == 16) return go(tridiag_back_kernel<4, 16>);
  if (c == 8) return go(tridiag_back_kernel<4, 8>);
  return go(tridiag_back_kernel<4, 4>);
}

}  // namespace itn
