/*
 * itn.h -- C ABI of libitn, a gfx950 (MI355X) implementation of the hot path
 * of two-site DMRG: the effective-Hamiltonian matvec H_eff*psi in dense and
 * quantum-number (QN) block-sparse form, the environment update, the labelled
 * contraction it is built from, and a sweep driver around them.
 *
 * Conventions shared by every call
 *  - Every call returns an itn_status and never throws.  Arguments are
 *    validated before any device work is queued; on a validation error no
 *    output is written.  itn_last_error() returns a message for the last
 *    failing call on a handle.
 *  - Tensors are row-major in the index order the call states (last index
 *    fastest).  Device data is caller-owned: the library never frees it and
 *    keeps no pointer to it after a call returns.
 *  - Launches are asynchronous and ordered on the hip stream passed in
 *    (NULL = the null stream).  Faults of queued kernels surface as
 *    ITN_E_HIP at the next call that synchronises, or at itn_sync().
 *  - The library owns its workspace (device scratch reused across calls and
 *    grown on demand), its QN plans and their captured hipGraphs.  A handle is
 *    not thread-safe; calls on one handle are serialised by the caller.
 *
 * Notation (the paper's MPS formula in Sec. 7.3, the operator element
 * convention op[s', s] of the hard-core boson example in Sec. 8.3):
 *   MPS site  A[a_{i-1}, s, a_i]           MPO site  W[m_{i-1}, m_i, s', s]
 *   left env  L[a', m, a]                   right env R[b', m, b]
 *   two-site  psi[a, s1, s2, b]
 *   (H_eff psi)[a', s1', s2', b'] =
 *      sum L[a', m0, a] W1[m0, m1, s1', s1] W2[m1, m2, s2', s2] R[b', m2, b] psi[a, s1, s2, b]
 * This is the local problem of the DMRG algorithm of Sec. 7.2 ("forming the
 * environment tensors and diagonalizing the local effective Hamiltonian");
 * the contraction strategy of Sec. 9.4 (permute to matrices, then GEMM) is
 * replaced here by MFMA kernels with the permutations folded into their
 * address maps.
 */
#ifndef ITN_H
#define ITN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ITN_OK = 0,
  ITN_E_ARG = 1,           /* null pointer, bad enum, bad count                         */
  ITN_E_SHAPE = 2,         /* extents inconsistent between operands                     */
  ITN_E_LABEL = 3,         /* labels repeated, or output labels != uncontracted labels  */
  ITN_E_ARROW = 4,         /* contracted QN indices with equal arrows (Sec. 8.2)        */
  ITN_E_FLUX = 5,          /* a block violating the flux rule, or flux mismatch (Sec. 8)*/
  ITN_E_DTYPE = 6,         /* dtype / precision combination not supported               */
  ITN_E_WORKSPACE = 7,     /* workspace allocation failed                               */
  ITN_E_HIP = 8,           /* a HIP / rocSOLVER call failed                             */
  ITN_E_NOT_CONVERGED = 9, /* eigensolver stopped above its tolerance (result kept)     */
  ITN_E_UNSUPPORTED = 10,  /* valid request the library does not implement              */
  ITN_E_NODEVICE = 11      /* compute call on a host-only handle                        */
} itn_status;

typedef enum { ITN_F64 = 0, ITN_F32 = 1, ITN_BF16 = 2 } itn_dtype; /* storage type */

/* Operand precision of the matrix-core contractions.  Accumulation is FP64
 * for ITN_P_F64 and FP32 otherwise; every operand is rounded to this type
 * before it enters an MFMA tile. */
typedef enum { ITN_P_F64 = 0, ITN_P_F32 = 1, ITN_P_BF16 = 2 } itn_prec;

typedef enum { ITN_LEFT = 0, ITN_RIGHT = 1 } itn_dir;

typedef struct itn_handle itn_handle;
typedef struct itn_plan itn_plan;
typedef struct itn_mps itn_mps;
typedef struct itn_mpo itn_mpo;

/* One QN index (Sec. 8.2): an ordered list of sectors, each a QN of nq
 * integer components and a dimension, and an arrow.  Host memory, read
 * during the call only.  Sectors with equal QNs may repeat. */
typedef struct {
  int32_t nsec;
  int32_t nq;
  const int32_t* qn;  /* nsec*nq, sector-major */
  const int32_t* dim; /* nsec */
  int8_t arrow;       /* +1 Out (QNs add to the flux), -1 In (subtract) */
  const int32_t* mod; /* nq addition rules, or NULL (all integer): 0 = integer
                         addition, N >= 2 = Z_N addition (values taken mod N;
                         Sec. 8).  Every index of every operand of one call
                         must use the same rules. */
} itn_space;

/* A tensor argument.
 *  dense   : nblocks == 0; dims[rank] gives the extents; data row-major.
 *  QN      : space[rank] gives the indices; blocks are the sector tuples
 *            block_sec[nblocks*rank] (0-based), sorted lexicographically with
 *            the first index most significant; block b starts at element
 *            block_off[b] of data and is row-major within itself; flux[nq] is
 *            the tensor's flux.  (Sec. 9.2 keeps one array plus a
 *            block->offset map; this layout fixes that map.)
 *  label   : integer index labels, used by itn_contract only (Sec. 9.1:
 *            equal labels are contracted, the rest survive).
 *  data    : device pointer (host pointer where a call says so). */
typedef struct {
  int32_t rank;
  const int64_t* dims;
  const int32_t* label;
  const itn_space* space;
  itn_dtype dtype;
  void* data;
  int64_t nblocks;
  const int32_t* block_sec;
  const int64_t* block_off;
  const int32_t* flux;
} itn_tensor;

/* ---------------------------------------------------------------- handle */

/* Create a handle on HIP device `device`.  device = -1 gives a host-only
 * handle that can validate arguments and build QN plans but returns
 * ITN_E_NODEVICE from any call that would launch work. */
itn_status itn_create(itn_handle** h, int device);
itn_status itn_destroy(itn_handle* h);
const char* itn_last_error(const itn_handle* h);
/* Wait for all work queued by the library on `hip_stream`; reports faults. */
itn_status itn_sync(itn_handle* h, void* hip_stream);
/* Library version string (static storage). */
const char* itn_version(void);

/* Per-kernel timing with hip events recorded on the launch stream around
 * each internal launch (small overhead per launch; off by default). */
itn_status itn_profile_enable(itn_handle* h, int32_t on);
/* Synchronise the device and report the launches timed since the last
 * report, aggregated by kernel name in first-seen order: names[32*i] (NUL-
 * terminated), total_ms[i], count[i] for i < min(*n_entries, max_entries).
 * Clears the record. */
itn_status itn_profile_report(itn_handle* h, int32_t max_entries, char* names, double* total_ms,
                              int64_t* count, int32_t* n_entries);

/* dst = src converted element-wise to dst's dtype (dense, equal extents;
 * F64 / F32 / BF16 both ways, rounding to nearest).  Used to prepare
 * environments in the matrix-core operand type once per bond. */
itn_status itn_cast(itn_handle* h, const itn_tensor* src, itn_tensor* dst, void* hip_stream);

/* ------------------------------------------------------------- workspace */

/* Operations whose scratch comes from the handle's workspace. */
typedef enum { ITN_OP_CONTRACT = 0, ITN_OP_HEFF = 1, ITN_OP_ENV_UPDATE = 2 } itn_op;

/* Bytes of workspace one call would use: `t` holds that call's tensors in
 * its argument order (ITN_OP_CONTRACT: A, B, C; ITN_OP_HEFF: L, W1, W2, R,
 * psi; ITN_OP_ENV_UPDATE: E, A, W, E_out), with nv (H_eff) and dir
 * (environment step) as the call takes them; data pointers are not read.
 * The arguments are validated exactly as the call does (same errors).
 * Host-only handles may ask. */
itn_status itn_workspace_size(itn_handle* h, itn_op op, int32_t ntensors, const itn_tensor* const* t,
                              int32_t nv, int32_t dir, itn_prec prec, size_t* bytes);

/* Use caller-owned device memory (256-byte aligned, `bytes` long) as the
 * handle's workspace from now on: the library then never grows it, and a
 * call needing more returns ITN_E_WORKSPACE before queuing work.  The
 * memory must stay allocated, and is not touched by anything else, while
 * calls on the handle may run; the library never frees it.  ptr = NULL
 * (bytes = 0) returns to library-owned workspace.  Waits for the device.
 * W-stage tables and QN plans stay library-owned. */
itn_status itn_set_workspace(itn_handle* h, void* ptr, size_t bytes);

/* --------------------------------------------------------------- contract */

/* C = A * B over labels (the product operator of Sec. 4 with the label
 * interface of Sec. 9.1): labels shared by A and B are summed; C's labels
 * must be exactly the remaining ones, in any order (the caller fixes the
 * output order).  No shared label is an outer product, all shared (rank-0
 * C) an inner product.  Dtypes F64 or F32 for A, B, C (ITN_P_BF16 rounds
 * operands to bf16).  Errors: ITN_E_LABEL, ITN_E_SHAPE, ITN_E_DTYPE.
 *
 * Block-sparse operands (all three carry `space`; Sec. 8, 9.4): every pair
 * of an A block and a B block whose contracted sectors agree is a dense
 * block product; pairs landing on one C block are summed in ascending
 * (A block, B block) order.  Contracted indices must have opposite arrows
 * (ITN_E_ARROW) and equal sectors (ITN_E_SHAPE); each C index keeps the
 * arrow and sectors of the index it comes from; every given block must obey
 * its tensor's flux rule and flux(C) must equal flux(A) + flux(B)
 * (ITN_E_FLUX).  C's block list must hold every block a contributing pair
 * reaches (ITN_E_FLUX otherwise); C blocks no pair reaches are set to zero.
 * All block products run as one grouped launch.  Mixing dense and
 * block-sparse operands is ITN_E_ARG. */
itn_status itn_contract(itn_handle* h, const itn_tensor* A, const itn_tensor* B, itn_tensor* C,
                        itn_prec prec, void* hip_stream);

/* ------------------------------------------------------------ dense H_eff */

/* out = H_eff * psi for nv vectors (dense).
 *  L   [chi_l, w, chi_l]   device, F64 / F32 / BF16
 *  W1  [w, w, d, d]        HOST, F64 (the MPO site tensors are tiny; the
 *  W2  [w, w, d, d]        HOST, F64  library derives per-pair tables)
 *  R   [chi_r, w, chi_r]   device, F64 / F32 / BF16
 *  psi [chi_l, d, d, chi_r] device, F64 / F32: nv vectors stored one after
 *       another (vector stride chi_l*d*d*chi_r elements)
 *  out same shape and stride as psi, F64 / F32, must not alias psi.
 * The contraction order is L first, then W1 W2 (fused into the first
 * stage's epilogue when w*d*d <= 48), then R.  Operands whose dtype differs
 * from `prec` are converted in workspace each call; pass L and R already in
 * the compute type to avoid it.  Errors: ITN_E_SHAPE, ITN_E_DTYPE, ITN_E_ARG. */
itn_status itn_heff_apply(itn_handle* h, const itn_tensor* L, const itn_tensor* W1,
                          const itn_tensor* W2, const itn_tensor* R, const itn_tensor* psi,
                          int32_t nv, itn_tensor* out, itn_prec prec, void* hip_stream);

/* out = sum over k < nterms of H_eff,k * psi: the effective Hamiltonian of a
 * sum of MPOs H = H_0 + H_1 + ... (Sec. 7.2, a Hamiltonian given as several
 * MPOs summed implicitly).  L[k], W1[k], W2[k], R[k] are one term's operands
 * with the layouts and dtypes of itn_heff_apply; each term may have its own
 * MPO bond dimension w_k, all share chi_l, chi_r, d and psi.  psi is
 * transposed once; every term's last stage adds into out (bit-identical to a
 * single itn_heff_apply for nterms = 1).  Arrays of nterms pointers, owned by
 * the caller.  Errors: as itn_heff_apply, and ITN_E_ARG for nterms < 1. */
itn_status itn_heff_apply_sum(itn_handle* h, int32_t nterms, const itn_tensor* const* L,
                              const itn_tensor* const* W1, const itn_tensor* const* W2,
                              const itn_tensor* const* R, const itn_tensor* psi, int32_t nv,
                              itn_tensor* out, itn_prec prec, void* hip_stream);

/* itn_heff_apply for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, kernels and results (bit-identical to itn_heff_apply), but
 * every scratch buffer of the call -- psi transposed, the W-stage output,
 * converted environments, the W-stage tables -- is carved from one fixed
 * device array of the library (itn_heff_noalloc_max_bytes, 64 MiB; enough
 * for chi_l = chi_r = 1024 at d = 2, w = 5, nv = 1 in bf16).  A request
 * needing more returns ITN_E_WORKSPACE with the size it needs, before any
 * work is queued.  The call allocates nothing: the W-stage tables are copied
 * into the array on the stream.  Each device holds its own array, shared by
 * every call on that device: calls that overlap on one device (other
 * streams, threads or handles) race and must be serialised by the caller. */
itn_status itn_heff_apply_noalloc(itn_handle* h, const itn_tensor* L, const itn_tensor* W1,
                                  const itn_tensor* W2, const itn_tensor* R, const itn_tensor* psi,
                                  int32_t nv, itn_tensor* out, itn_prec prec, void* hip_stream);
/* Size in bytes of that fixed scratch array. */
itn_status itn_heff_noalloc_max_bytes(size_t* bytes);

/* Bytes of library workspace itn_heff_apply uses for these extents (the
 * upper bound; itn_workspace_size gives the exact figure of one call). */
itn_status itn_heff_workspace_size(itn_handle* h, int64_t chi_l, int64_t chi_r, int32_t d,
                                   int32_t w, int32_t nv, itn_prec prec, size_t* bytes);

/* -------------------------------------------------------------- QN H_eff */

/* Build the plan of a block-sparse H_eff*psi (Sec. 8, Sec. 9.4): from the
 * sector tables of L[a':Out, m:In, a:In], W1/W2[m_in:Out, m_out:In, s':Out,
 * s:In], R[b':In, m:Out, b:Out] and psi[a:Out, s1:Out, s2:Out, b:In] it
 * enumerates the allowed blocks by the flux rule, checks that every given
 * block is allowed (ITN_E_FLUX) and that contracted indices have opposite
 * arrows and equal sectors (ITN_E_ARROW, ITN_E_SHAPE), groups the block
 * products by contracted sector pair, and fixes the order in which
 * contributions to one output block are summed.  Integer host work only: a
 * host-only handle may plan.  W1/W2 data are HOST F64 dense [w,w,d,d].
 * The plan stores copies of everything it needs. */
itn_status itn_qn_heff_plan(itn_handle* h, const itn_tensor* L, const itn_tensor* W1,
                            const itn_tensor* W2, const itn_tensor* R, const itn_tensor* psi,
                            int32_t nv, itn_prec prec, itn_plan** plan);
itn_status itn_plan_destroy(itn_plan* plan);

/* Plan queries (host).  Output block structure of H_eff*psi: the sector
 * tuples and offsets (same layout as itn_tensor), and the work figures. */
typedef struct {
  int64_t out_nblocks;     /* number of output blocks (equals psi's)              */
  int64_t out_elems;       /* elements per vector                                 */
  int64_t n_pairs_stage1;  /* block pairs L x psi                                 */
  int64_t n_groups_stage1; /* L x psi products: one per a-sector (all m0 stacked) */
  int64_t n_pairs_stage4;  /* K segments of the Z x R products (one product per   */
                           /* b'-sector, one segment per (m2, b) sector pair)      */
  int64_t n_tiles;         /* work items of the grouped launches                  */
  double flops;            /* 2*M*N*K summed over contributing block products, x nv */
  int64_t x_elems;         /* stage-1 intermediate X, elements per vector (not    */
                           /* counting the zero columns that pad each b-sector    */
                           /* to a multiple of 8)                                 */
  int64_t z_elems;         /* W-stage output Z (stage-4 operand), per vector, ditto */
  double flops_wstage;     /* 2 * W12 terms * positions, x nv (not in flops)      */
  int32_t mode_stage1;     /* grouped launch modes of stages 1 and 4 (0..7, see   */
  int32_t mode_stage4;     /* itn_qn_heff_apply); -1 before the first apply       */
  int32_t wstage_tile;     /* W-stage work item: 16-byte vectors per wave (64,    */
                           /* 128 or 256); -1 before the first apply              */
  double flops_stage1;     /* the part of `flops` in the L*psi stage (the rest is   */
                           /* the Z*R stage)                                         */
} itn_plan_info;
itn_status itn_plan_query(const itn_plan* plan, itn_plan_info* info);
/* Copy the output block table: block_sec[out_nblocks*4], block_off[out_nblocks]. */
itn_status itn_plan_out_blocks(const itn_plan* plan, int32_t* block_sec, int64_t* block_off);

/* Enumerate the allowed blocks of a QN tensor's indices (t->space, t->rank,
 * t->flux; NULL flux = zero): the sector tuples whose Out QNs minus In QNs
 * equal the flux (Sec. 8), in the packing order of itn_tensor, with their
 * offsets.  Call with block_sec == NULL to get *nblocks and *total only;
 * otherwise block_sec[*nblocks * rank] and block_off[*nblocks] are filled
 * (their capacity is the *nblocks passed in).  Host-only handles may call. */
itn_status itn_qn_allowed_blocks(itn_handle* h, const itn_tensor* t, int64_t* nblocks,
                                 int32_t* block_sec, int64_t* block_off, int64_t* total);

/* Apply a plan.  Tensors must carry the same sector tables and block lists
 * the plan was built from (checked by signature: ITN_E_SHAPE otherwise);
 * data pointers may change between calls.  psi/out hold nv vectors at stride
 * out_elems.  The first call on a stream captures the launches into a
 * hipGraph that later calls replay.
 * The first apply also picks, per grouped stage, the fastest launch mode by
 * timing them on the real operands (0: 64x64 tiles; 1: 128x128; 2, 3: block
 * products with both extents >= 192 on 256-row direct-to-LDS tiles, the rest
 * on 64 / 128; 4: as 2, with the remaining products of both extents >= 96
 * on 128x128 direct-to-LDS tiles; 5: products of both extents >= 96 on
 * 128x128 direct-to-LDS tiles, the rest on 64; 6: as 5, with the products
 * of M >= 96 and N < 96 on 256x64 direct-to-LDS tiles; 7: as 4, with those
 * narrow products on 256x64 direct-to-LDS tiles).  The choice is cached per
 * operand structure (in the file ITN_AUTOTUNE_CACHE if set);
 * ITN_QN_TILE_MODE="m1,m4" (modes 0..7) fixes it instead.
 * L == NULL and R == NULL apply with the environments of the last
 * itn_qn_prepare_env (or of the last apply that passed them) without
 * repacking them again (ITN_E_ARG if there are none); passing only one of
 * them is ITN_E_ARG. */
itn_status itn_qn_heff_apply(itn_handle* h, itn_plan* plan, const itn_tensor* L,
                             const itn_tensor* R, const itn_tensor* psi, itn_tensor* out,
                             void* hip_stream);

/* Diagonal of the block-sparse two-site H_eff (the operands of
 * itn_qn_heff_plan, Sec. 7.2 with Sec. 8): out[a, s1, s2, b] = sum over m0,
 * m1, m2 of L[a, m0, a] W1[m0, m1, s1, s1] W2[m1, m2, s2, s2] R[b, m2, b],
 * the preconditioner of block Davidson.  L, R: device F64 block-sparse (any
 * flux-allowed block lists); W1, W2: host F64 dense with their QN spaces;
 * out: device F64, psi's index spaces and arrows, every listed block written.
 * Only zero-charge MPO channels reach the diagonal (the environments' flux
 * rule).  Uses the handle's workspace (small: the environments' diagonals
 * and the block tables) and returns after the work on hip_stream has
 * finished.  Errors: ITN_E_ARROW, ITN_E_SHAPE (sectors differ), ITN_E_DTYPE,
 * ITN_E_FLUX, ITN_E_WORKSPACE, ITN_E_NODEVICE. */
itn_status itn_qn_heff_diag(itn_handle* h, const itn_tensor* L, const itn_tensor* W1,
                            const itn_tensor* W2, const itn_tensor* R, itn_tensor* out,
                            void* hip_stream);

/* Repack the environments L, R (the plan's structure and compute type:
 * ITN_E_SHAPE / ITN_E_DTYPE otherwise) into the plan's layouts on
 * hip_stream, for applies with L = R = NULL.  The eigensolver at a bond of
 * a DMRG sweep (Sec. 7.2) applies H_eff many times with the same
 * environments: their repack is then paid once per bond, not per apply.
 * L and R must stay unchanged and allocated while such applies run. */
itn_status itn_qn_prepare_env(itn_handle* h, itn_plan* plan, const itn_tensor* L,
                              const itn_tensor* R, void* hip_stream);

/* ------------------------------------------------------- environment step */

/* One environment step (Sec. 7.2, "forming the environment tensors").
 *  dir = ITN_LEFT :  E_out[a', m', a] = sum E[a'', m, a'''] A[a'', s', a'] W[m, m', s', s] A[a''', s, a]
 *  dir = ITN_RIGHT:  E_out[b', m, b]  = sum A[b', s', b''] W[m, m', s', s] A[b, s, b'''] E[b'', m', b''']
 *  E [chi, w, chi] device; A [chi_l, d, chi_r] device; W [w, w, d, d] HOST F64;
 *  E_out device.  Dense; dtypes F64 / F32 (E, A, E_out). */
itn_status itn_env_update(itn_handle* h, const itn_tensor* E, const itn_tensor* A,
                          const itn_tensor* W, itn_dir dir, itn_tensor* E_out, itn_prec prec,
                          void* hip_stream);

/* ------------------------------------------------------------ DMRG sweeps */

/* MPO of N sites, all with the same w and d: W_host holds N tensors
 * [w, w, d, d] (F64) back to back.  Lower-triangular boundary convention:
 * the left boundary selects channel w-1, the right boundary channel 0. */
itn_status itn_mpo_create(itn_handle* h, int32_t N, int32_t w, int32_t d, const double* W_host,
                          itn_mpo** mpo);
itn_status itn_mpo_destroy(itn_mpo* mpo);

/* MPS of N sites (F64, device-resident inside the object).  bond[N+1] gives
 * the link dimensions (bond[0] = bond[N] = 1); sites_host holds the N site
 * tensors [bond[i], d, bond[i+1]] back to back.  The state must be
 * right-canonical with its norm on site 0 (a normalised product state is). */
itn_status itn_mps_create(itn_handle* h, int32_t N, int32_t d, const int32_t* bond,
                          const double* sites_host, itn_mps** mps);
itn_status itn_mps_destroy(itn_mps* mps);
/* Current link dimensions (N+1 entries). */
itn_status itn_mps_bonds(const itn_mps* mps, int32_t* bond);
/* Copy site i to host ([bond[i], d, bond[i+1]] doubles). */
itn_status itn_mps_get_site(itn_handle* h, const itn_mps* mps, int32_t i, double* host);

typedef struct {
  int32_t nsweeps;
  const int32_t* maxdim;  /* nsweeps entries (the Sweeps schedule of Sec. 7.2) */
  const double* cutoff;   /* nsweeps entries (truncation of Sec. 5)            */
  int32_t mindim;         /* >= 1                                              */
  int32_t krylovdim;      /* Davidson basis size before restart (>= 2)        */
  int32_t maxiter;        /* matvecs per local eigensolve                      */
  double eig_tol;         /* residual tolerance, relative to |theta|           */
  itn_prec prec;          /* matvec precision of the Davidson expansion        */
  int32_t refine;         /* with prec below F64, 1: apply the first vector of
                             every restart cycle in FP64 (exact couplings to
                             the low-precision corrections; the solve converges
                             to the FP64 eigenpair), 0: every matvec at prec  */
  double energy_tol;      /* stop early when |dE| < energy_tol*|E| (0: never)  */
  int32_t timing;         /* 1: synchronise at phase boundaries and report the
                             per-phase times below (adds host waits)           */
  /* Excited states (Sec. 7.2): previously found states whose projectors,
   * times the energy penalty `weight`, are added to the Hamiltonian, so the
   * sweep converges to the lowest state orthogonal to them when the weight
   * exceeds the gap.  ortho: northo MPS handles with the same N and d (not
   * the MPS being optimised), read only; northo = 0: none. */
  int32_t northo;
  const itn_mps* const* ortho;
  double weight;
  /* Block size of the Davidson expansion: each step adds the residuals of
   * the `block` lowest Ritz pairs and applies H_eff to them in one batched
   * itn_heff_apply (itn_qn_heff_apply on block-sparse sweeps; nv = block,
 * at most 8).  0 or 1: one vector per step. */
  int32_t block;
} itn_sweep_params;

/* Per-sweep results, arrays of nsweeps entries owned by the caller (any may
 * be NULL).  sweeps_done is set to the number of sweeps actually run. */
typedef struct {
  int32_t sweeps_done;
  double* energy;       /* eigenvalue at the last bond of the sweep            */
  double* max_trunc;    /* largest discarded weight of the sweep               */
  int32_t* max_bond;    /* largest link dimension after the sweep              */
  double* seconds;      /* wall time of the sweep                              */
  int64_t* matvecs;     /* H_eff applications in the sweep (all precisions)    */
  double* residual;     /* largest final FP64 residual norm of a local solve   */
  /* Per-phase seconds of the sweep, filled when params->timing is 1 (any may
   * be NULL): H_eff applications; the rest of the local eigensolves (basis
   * BLAS-1, projected problem, restarts); bond splits; environment updates. */
  double* t_matvec;
  double* t_solver;
  double* t_split;
  double* t_env;
  int64_t* matvecs_f64; /* of `matvecs`, those applied in FP64                 */
} itn_sweep_result;

/* Run the schedule: per sweep, left->right over bonds (0,1)..(N-2,N-1) then
 * right->left back (two-site updates, truncated split of Sec. 5, FP64
 * eigensolver).  The MPS and its environments are updated in place, so a
 * later call continues where this one stopped.  Returns
 * ITN_E_NOT_CONVERGED (after finishing the sweeps) if a local solve ended
 * above its tolerance. */
itn_status itn_dmrg_sweep(itn_handle* h, itn_mps* mps, const itn_mpo* mpo,
                          const itn_sweep_params* params, itn_sweep_result* result);

/* ------------------------------------------------- block-sparse DMRG sweeps */

/* A block-sparse MPS (Sec. 8, 9.2): every site tensor A[a:Out, s:Out, a':In]
 * holds only its flux-allowed blocks; the link charge is the total QN of the
 * sites to its left, so the state has the definite total QN of its last link.
 * Created as the product state state[i] (basis index per site; Neel states
 * fix the sector).  site_qn[d*nq] gives the QN of each basis state (runs of
 * equal QN form one sector), mod[nq] the addition rules (NULL: integer). */
typedef struct itn_qn_mps itn_qn_mps;
itn_status itn_qn_mps_create(itn_handle* h, int32_t N, int32_t d, int32_t nq, const int32_t* site_qn,
                             const int32_t* mod, const int32_t* state, itn_qn_mps** mps);
itn_status itn_qn_mps_destroy(itn_qn_mps* mps);
/* Total link dimensions (N+1 entries). */
itn_status itn_qn_mps_bonds(const itn_qn_mps* mps, int32_t* bond);
/* Link k's sectors: on entry *nsec is the capacity of qn[*nsec*nq] and
 * dim[*nsec] (NULL arrays: query only); on return the number of sectors. */
itn_status itn_qn_mps_link(const itn_qn_mps* mps, int32_t k, int32_t* nsec, int32_t* qn, int32_t* dim);
/* Site i as a dense host array [bond[i], d, bond[i+1]] (blocks embedded at
 * their sector offsets, zero elsewhere). */
itn_status itn_qn_mps_get_site(itn_handle* h, const itn_qn_mps* mps, int32_t i, double* host);

/* Two-site DMRG sweeps on a block-sparse MPS (Sec. 7.2 with Sec. 8):
 * link_qn[w*nq] gives the QN each MPO channel carries (W[m_in:Out, m_out:In,
 * s':Out, s:In] with zero flux; a nonzero MPO entry outside the allowed
 * blocks is ITN_E_FLUX).  At each bond the local problem is the planned
 * block-sparse H_eff (itn_qn_heff_plan), the eigensolver that of
 * itn_dmrg_sweep (precision, refinement and block as there: with block > 1
 * the plans carry `block` vectors per launch and the preconditioner is the
 * block-sparse H_eff diagonal; no excited states: ITN_E_UNSUPPORTED), and
 * the bond is split per charge sector of the new
 * link: each sector's density matrix is diagonalised and the truncation of
 * Sec. 5 is applied to the weights of all sectors together; environments are
 * block-sparse contractions.  The total QN is conserved exactly. */
itn_status itn_qn_dmrg_sweep(itn_handle* h, itn_qn_mps* mps, const itn_mpo* mpo, const int32_t* link_qn,
                             const itn_sweep_params* params, itn_sweep_result* result);

#ifdef __cplusplus
}
#endif
#endif /* ITN_H */
