// Host-callable launchers of the engine's HIP kernels.
#pragma once

#include <vector>

#include "common.hpp"

namespace ttnn {

// ---------------------------------------------------------------- DRMs
void launch_drm(int64_t rows, int cols, uint64_t seed, uint32_t tag, double* o64, float* o32,
                uint16_t* o16, hipStream_t stream);
// The n x n identity (the maps of a free mode) in FP64 and, where given, FP32 / BF16.
void launch_eye(int64_t n, double* o64, float* o32, uint16_t* o16, hipStream_t stream);

// ---------------------------------------------------------------- generic contraction
// The operand H (dtype th) is viewed as [L][n][Q] column-major (L fastest) and as the
// matrix Hm(m, i) with m = l + L q:  Hm(m, i) = H[l + L (i + n q)].
//   RIGHT: out(c; i, j) = sum_{m in chunk c} Hm(m, i) D(drow(m), j),
//          drow(m) = amap(m % L) + bmap(m / L)
//   LEFT : out(c; m, j) = sum_{i in chunk c} Hm(m, i) D(drow(i), j),  drow(i) = amap(i)
// D(row, j) = D[row * sDr + j * sDc] (dtype td).  Results are FP64 (or FP32 when
// out_f32) stored at  out[c*cs + (row % Lo)*s0 + j*s1 + (row / Lo)*s2].
struct OutLayout {
  int64_t Lo, s0, s1, s2, cs;
};

// Address of entry (l, i, q) of the operand H[L][n][Q]: packed, l + L (i + n q); or,
// for a box read in place from a strided array (the caller's tensor), the sum of three
// position maps over the box positions before the contracted group (ml), the group
// (mi) and the positions after it (mq), each with the caller's element strides.
struct HMap {
  int32_t strided = 0, pad_ = 0;
  IndexMap ml, mi, mq;
  __host__ __device__ inline int64_t operator()(int64_t l, int64_t i, int64_t q, int64_t L, int64_t n) const {
    return strided ? ml(l) + mi(i) + mq(q) : l + L * (i + n * q);
  }
};

struct GemmArgs {
  bool right = true;
  const void* H = nullptr;
  int th = TTNN_F64;
  int64_t L = 1, n = 1, Q = 1;
  const void* D = nullptr;
  int td = TTNN_F64;
  int64_t sDr = 1, sDc = 1;
  int ncols = 1;
  IndexMap amap, bmap;
  HMap hm;                     // operand addressing (packed unless a strided raw box)
  int nchunks = 1;
  void* out = nullptr;
  bool out_f32 = false;
  OutLayout ol{};
};
// Returns the number of chunks actually written (<= a.nchunks); 0 if nothing to do.
int launch_gemm(const GemmArgs& a, hipStream_t stream);

// choose the split over the contraction index; returns the number of chunks
int pick_chunks(int64_t rows, int ncols, int64_t K, size_t partial_cap);
// The number of chunks launch_gemm writes for `a` (0 if nothing to do) and their length.
int gemm_chunks(const GemmArgs& a, int64_t* kchunk);

// ---------------------------------------------------------------- batched launches
// Descriptors as the batched kernels read them (device memory, staged per launch).
struct GemmTask {
  const void* H;
  const void* D;
  void* out;
  int64_t L, n, Q, sDr, sDc, kchunk;
  int64_t row_blocks, nch, col_blocks, first_block;
  IndexMap amap, bmap;
  HMap hm;
  OutLayout ol;
  int32_t ncols, pad_;
};
struct ReduceTask {
  double* part = nullptr;
  double* dst = nullptr;
  int64_t rows = 0, ldr = 0, L = 1, kdim = 1;
  double alpha = 1.0;
  IndexMap rmap;
  int64_t first_block = 0, nblocks = 0;
  int64_t cstride = 0;                     // distance between chunk partials (0: rows * ncols)
  int32_t nchunks = 0, ncols = 0, mode = 0, groups = 0;
};
// Launch the same kind of generic contraction (right/left, dtypes, output type) for
// every element of `args` in one kernel: each workgroup serves one tile of one task.
// Results are bitwise those of launch_gemm on each element.
void launch_gemm_batched(const std::vector<GemmArgs>& args, hipStream_t stream);
// Fixed-order partial sums of several contractions in one launch (see launch_reduce).
void launch_reduce_batched(const std::vector<ReduceTask>& tasks, hipStream_t stream);
// The same two launches split into building the descriptor tables on the host and
// launching from tables already staged on the device, so that a caller can stage the
// tables of many launches in one copy.
struct BatchedGemm {
  std::vector<GemmTask> tasks;
  int64_t blocks = 0;
  bool right = true, out_f32 = false;
  int th = TTNN_F64, td = TTNN_F64;
};
BatchedGemm plan_gemm_batched(const std::vector<GemmArgs>& args);
void launch_gemm_staged(const BatchedGemm& b, const GemmTask* d_tasks, hipStream_t stream);
struct BatchedReduce {
  std::vector<ReduceTask> folds, tasks;
  int64_t fblocks = 0, blocks = 0;
};
BatchedReduce plan_reduce_batched(const std::vector<ReduceTask>& tasks);
void launch_reduce_staged(const BatchedReduce& b, const ReduceTask* d_folds, const ReduceTask* d_tasks,
                          hipStream_t stream);
// Persistent ingest: every phase of a batched round of box updates in one cooperative
// launch (level by level: the contractions of all kinds, the chunk folds, the
// reductions; grid-wide barriers between phases), bitwise the same results as the
// per-level launches.  gl / level_end / rl as built for those launches (all plans of
// compute dtype cd); sticky: each plan's sticky status word (set if a barrier wait ran
// out).  Returns false, launching nothing, when the round does not fit the program
// (too many phases, segments or plans, FP32 outputs) or the device cannot launch it.
constexpr int kIngestSegs = 4, kIngestPlans = 128, kIngestPhases = 48;
enum : int32_t { kSegRightRaw = 0, kSegLeftRaw = 1, kSegRightF64 = 2, kSegLeftF64 = 3, kSegFold = 4, kSegReduce = 5 };
bool launch_ingest(int cd, const std::vector<BatchedGemm>& gl, const std::vector<size_t>& level_end,
                   const std::vector<BatchedReduce>& rl, const std::vector<int*>& sticky, hipStream_t stream);
// Copy `bytes` of host descriptors into device memory that stays valid for work
// enqueued on `stream` after this call and before the next fence_descriptors on it
// (pinned staging ring, reused once the fenced work has finished).
void* stage_descriptors(const void* host, size_t bytes, hipStream_t stream);
// Mark the end of the work that reads the descriptors staged so far on `stream`.
void fence_descriptors(hipStream_t stream);
// Held from staging to fence, so that another host thread cannot wrap the ring in between.
struct StagingLock {
  StagingLock();
  ~StagingLock();
  StagingLock(const StagingLock&) = delete;
  StagingLock& operator=(const StagingLock&) = delete;
};

// Sum partial results over chunks in a fixed order (FP64) and deliver them.
//   mode 0 (RIGHT accumulate): dst[rmap(row) + ldr*j] += alpha * s
//   mode 1 (LEFT  accumulate): dst[(row % L) + L*(j + kdim*(row / L))] += alpha * s
//   mode 2 (LEFT  store)     : dst[(row % L) + L*(j + kdim*(row / L))]  = s
// With many chunks and few elements the partials are first folded in place (groups of
// consecutive chunks, fixed order), so `part` is overwritten.
void launch_reduce(double* part, int nchunks, int64_t rows, int ncols, int mode, double alpha,
                   const IndexMap& rmap, int64_t ldr, double* dst, int64_t L, int64_t kdim,
                   hipStream_t stream);

// ---------------------------------------------------------------- batched FP64 GEMM
// C[cb](m,n) = (accumulate ? C : 0) + alpha * sum_{kb<nbK} sum_{k<K} A(m,k;cb,kb) B(k,n;cb,kb)
// with A(m,k;cb,kb) = A[m sAm + k sAk + cb sAc + kb sAkb] and likewise for B and C.
struct GJob {
  int64_t M = 0, N = 0, K = 0;
  int nbK = 1, nbC = 1;
  const double* A = nullptr;
  int64_t sAm = 0, sAk = 0, sAkb = 0, sAc = 0;
  const double* B = nullptr;
  int64_t sBk = 0, sBn = 0, sBkb = 0, sBc = 0;
  double* C = nullptr;
  int64_t sCm = 0, sCn = 0, sCc = 0;
  double alpha = 1.0;
  int accumulate = 0;
  // filled by the launcher
  int splits = 1;
  int64_t tiles_m = 0, tiles_n = 0, first_block = 0, first_tile = 0;
  double* part = nullptr;
};
constexpr int kMaxGJobs = 12;
struct GJobList {
  GJob jobs[kMaxGJobs];
  int n;
};
// Launches every job (in chunks of kMaxGJobs per kernel, plus one combine launch for
// the chunk's split contractions); `part` is split-contraction scratch.
void launch_bgemm64(std::vector<GJob>& jobs, double* part, size_t part_elems, hipStream_t stream);

// ---------------------------------------------------------------- rank-1 updates
// Kronecker vector over positions (first fastest): entry(row) = prod_p v[p][digit_p(row)].
struct KronVec {
  int n = 0;
  const double* v[kMaxPos] = {};
  int64_t len[kMaxPos] = {};
  void push(const double* p, int64_t l) {
    v[n] = p;
    len[n] = l;
    ++n;
  }
};
// Copy of a strided box (element strides per mode) into dst, packed column-major over
// ext (first mode fastest); dtype dt, d modes.
struct PackDims {
  int64_t ext[TTNN_MAX_ORDER] = {};
  int64_t stride[TTNN_MAX_ORDER] = {};
};
void launch_pack_box(const void* src, int dt, int d, const int64_t* ext, const int64_t* strides, void* dst,
                     hipStream_t stream);
// Strided boxes of at least this many entries are packed before their update.
constexpr int64_t kPackMinEntries = int64_t(1) << 22;

// Up to kRank1Batch rank-1 terms handled by one launch (their vectors and scales).
constexpr int kRank1Batch = 16;
struct KronBatch {
  int m = 0;
  KronVec kv[kRank1Batch];
  double alpha[kRank1Batch] = {};
  void push(const KronVec& k, double a = 1.0) {
    kv[m] = k;
    alpha[m] = a;
    ++m;
  }
};
// w[y * wstride + j] = sum_row D[row * ncols + j] * kv_y(row) for every term y < kb.m,
// D row-major rows x ncols of dtype dt (products and sums in FP64); deterministic
// (fixed blocks, fixed summation order), and each term's result is bitwise the same
// whatever the batch it is computed in.  The blocks of the terms over one chunk of rows
// run side by side on one XCD, so the chunk comes from HBM about once per batch.
// `partial` is scratch.
// grouped: the term-group form on the FP64 MFMA where the map's shape allows it (the
// caller keeps one choice for all of a plan's terms).
void launch_kron_gemv(const void* D, int dt, int64_t rows, int ncols, const KronBatch& kb, double* partial,
                      size_t partial_elems, double* w, int64_t wstride, bool grouped, hipStream_t stream);
// R[i + n j] += alpha_y * ku_y(i) * (w ? w[y * wstride + j] : 1) for y = 0 .. m-1 in that
// order, R column-major n x ncols (each entry sees the terms' additions in order, as
// with one launch per term).
void launch_outer_acc(double* R, int64_t n, int ncols, const KronBatch& ku, const double* w, int64_t wstride,
                      hipStream_t stream);

// ---------------------------------------------------------------- whole-tensor right sketch on MFMA
// H (dtype dt) viewed as [L][n][Q] (l fastest); Xt is the transposed DRM copy (r x m,
// m = L Q, contraction index contiguous).  Writes FP64 chunk partials
// part[(c n + i) r + j] and returns the number of chunks (sum them with launch_reduce);
// the chunks are as many as part_elems holds, so with part_elems = n r the single
// chunk is the result itself.  Throws if part_elems < n r.
bool right_mfma_eligible(int64_t L, int64_t n, int64_t Q, int r, int dt);

// Mode product of a packed whole tensor H[L][n][Q] (dtype dt, FP32 or FP64) with a
// map Y (n x k row-major, same dtype) at a group past mode 1, on MFMA:
// out[l + L (j + k q)] = sum_i H[l + L i + L n q] Y[i][j] (FP64).  Eligible: L > 1 a
// multiple of the 16-byte vector, k <= 128, and at least 32768 rows L Q.
bool mid_mfma_eligible(int64_t L, int64_t n, int64_t Q, int k, int dt);
void launch_mid_mfma(const void* H, int dt, int64_t L, int64_t n, int64_t Q, const void* Y, int k, double* out,
                     hipStream_t st);
// Split of such a right sketch over its contraction (pure host arithmetic): nch chunks
// of kchunk values, each writing an n x r FP64 partial, nch * n * r <= part_elems.
// Throws TTNN_E_INVALID when the shape is not covered or part_elems cannot hold one
// chunk.  cus: compute units of the device.
struct RightMfmaSplit {
  int64_t nch, kchunk;
};
RightMfmaSplit right_mfma_split(int64_t L, int64_t n, int64_t Q, int r, int dt, size_t part_elems, int cus);
// Where the head of a contraction chain (Y_g^T on the raw tensor, group g at mode 1,
// Q rows of k values) writes: through the partial scratch and a reduction while two
// chunks fit it, else as one chunk straight into the chain buffer of Q * k values.
inline bool chain_head_in_place(int64_t Q, int k, size_t partial_elems) {
  return 2 * static_cast<size_t>(Q) * static_cast<size_t>(k) > partial_elems;
}
int launch_right_mfma(const void* H, int dt, int64_t L, int64_t n, int64_t Q, const void* Xt, int64_t m, int r,
                      double* part, size_t part_elems, hipStream_t stream);

// out[i0 + d0 (i1 + d1 i2)] = round_dt(src[i0 s0 + i1 s1 + i2 s2]) where the coordinate
// `cdim` is below `lim`, else 0 (layout copies of the DRMs, rounded like the compute copies).
void copy_layout(const double* src, void* out, int dt, int64_t d0, int64_t d1, int64_t d2, int64_t s0, int64_t s1,
                 int64_t s2, int cdim, int64_t lim, hipStream_t stream);

// ---------------------------------------------------------------- small utilities
void launch_zero(double* p, int64_t n, hipStream_t stream);
// Several FP64 arrays in one launch: zero them, or set *flag when one holds a non-finite value.
struct SegList {
  static constexpr int kMax = 2 * TTNN_MAX_NODES + 1;    // two arrays per node plus the root's
  double* p[kMax];
  int64_t n[kMax];
  int count = 0;
  void push(double* ptr, int64_t len) {
    TTNN_REQUIRE(count < kMax, TTNN_E_INVALID, "too many arrays in one list launch");
    p[count] = ptr;
    n[count] = len;
    ++count;
  }
};
void launch_zero_list(const SegList& s, hipStream_t stream);
void launch_finite_list(const SegList& s, int* flag, hipStream_t stream);
void launch_axpy(double* y, const double* x, double alpha, int64_t n, hipStream_t stream);
void launch_copy_f64(double* dst, const double* src, int64_t n, hipStream_t stream);
void launch_f64_to_f32(float* dst, const double* src, int64_t n, hipStream_t stream);
void launch_finite_check(const double* p, int64_t n, int* flag, hipStream_t stream);
void launch_zero_int(int* p, int64_t n, hipStream_t stream);

// ---------------------------------------------------------------- recovery phase
// One workgroup per job: Householder QR of Omega (k x r, column-major), sign fix
// diag(R) >= 0, one-sided Jacobi SVD of R, eps-truncated pseudo-inverse.
struct QrJob {
  const double* Om;   // k x r
  double* Q;          // k x r out
  double* Pinv;       // r x r out
  int k, r;
  int slot;           // its kept-count entry d_kept[slot] (the launcher may split the list)
};
struct QrJobList {
  QrJob jobs[TTNN_MAX_NODES];
  int n;
};
// Jobs with 32 < r <= 64 and k <= 64, or k <= 96, run in kernels of their own (4 lanes
// per column), the others in the kernel of the narrower register paths and the LDS path.
// Each launch takes the dynamic LDS of its largest job (qr_pinv_lds_bytes).
void launch_qr_pinv(const QrJobList& jl, double eps_factor, int* d_kept, hipStream_t stream);
// Dynamic LDS of one job: Omega (then reflectors and R) and Q, (k | 1) x r doubles each.
size_t qr_pinv_lds_bytes(int k, int r);
// Whether a job with these k >= r fits the recovery kernel (one workgroup, its LDS);
// plans check every node at creation.
bool qr_pinv_fits(int k, int r);
// Status of one assembly from its flags (flags[0] non-finite count, flags[1..nn-1] kept
// singular values per node): *call = 1 if bad else 0, and *sticky |= *call.
void launch_status_fold(const int* flags, int nn, int* call, int* sticky, hipStream_t stream);

// ---------------------------------------------------------------- norms
// Deterministic two-pass sums of (a - b)^2 and b^2; result in d_out[0..1].
void launch_diff_norms(const void* a, int a_dtype, const double* b, int64_t n, double* d_part,
                       double* d_out, hipStream_t stream);
constexpr int kNormBlocks = 1024;
// The same two kernels with their 2 x kNormBlocks partials in a static device array
// (no allocation); d_out: two doubles of device memory, written in stream order.
void launch_diff_norms_static(const void* a, int a_dtype, const double* b, int64_t n, double* d_out,
                              hipStream_t stream);

}  // namespace ttnn
