/*
 * ttnn.h -- C ABI of the MI355X sketching engine for the tree tensor network
 * Nystrom method (TTNN) and its sequential variant (STTNN).
 *
 * Paper: A. Bucci, G. Verzella, "Randomized algorithms for streaming low-rank
 * approximation in tree tensor network format" (arXiv 2412.06111).
 *
 *   problem statement ........ Sec. 4, first paragraph, and the inputs of Alg. 2:
 *                              tensor of size n_1 x ... x n_d, index tree, TTN
 *                              ranks r_t and oversamples p_t (Sec. 4, eq. "sketch")
 *   sketch phase ............. Sec. 4 ("Sketch phase"): Omega_t = Y_t^T T^{t} X_t,
 *                              Psi_t for root / internal / leaf nodes
 *   sequential variant ....... Sec. 5 (projections on contracted tensors, node order)
 *   recovery phase ........... Sec. 4 ("Recovery phase"), Alg. 2, stabilised
 *                              least squares with eps = 10 u ||R||_2
 *   streaming ................ Sec. 4, paragraph after the recovery phase: the
 *                              sketches of T = sum_i lambda_i H_i are the sums of
 *                              the sketches of the H_i
 *   TTN format ............... Def. 5 and its matricised form (reconstruction)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Layout: every dense tensor is column-major, mode 1 fastest: entry
 *    (i_1, ..., i_d) (0-based) sits at sum_mu i_mu prod_{nu<mu} n_nu.  This is the
 *    index order of the matricisation of Def. 2.  A C-contiguous array of shape
 *    (n_d, ..., n_1) has exactly this layout.
 *  - Pointers named d_* are HIP device pointers; everything else is host memory.
 *    `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *  - Node ids in the ABI are the caller's ids: the positions in the parent[] /
 *    first_mode[] / last_mode[] arrays of the problem.  Internally the library
 *    renumbers nodes level by level, left to right (the labels of Fig. 1); that
 *    level-order id is the one that seeds the node's DRMs.
 *  - Asynchrony: calls enqueue work on `stream` and return.  Argument checks are
 *    done on the host before anything is enqueued and are reported synchronously.
 *    A failed HIP call makes the plan's status sticky (TTNN_E_HIP): later calls on
 *    that plan return it until ttnn_reset.  Input buffers must stay valid until
 *    the stream has passed the call.  A whole-tensor update may run part of its
 *    work on a side stream that the plan owns (default priority); that work starts
 *    after everything enqueued before the call on `stream` and is joined back into
 *    `stream` before the call returns, so ordering on `stream` is as if all of it
 *    ran there.
 *  - Ownership: the caller owns every buffer it passes.  A plan made by ttnn_plan
 *    lives in a device workspace the caller owns (ttnn_workspace_bytes gives its
 *    size): every device array of the plan (DRMs, FP64 accumulators, scratch) is a
 *    view into it, and the plan never frees it.  ttnn_plan_create instead takes one
 *    block from the library's per-device pool (stream ordered on its stream: use the
 *    plan on other streams only after that stream has passed the call), released by
 *    ttnn_destroy or ttnn_destroy_async.  ttnn_footprint_bytes reports the size.
 *    Besides plans the library keeps, per process, a small pinned/device ring that
 *    stages the descriptor tables of batched launches.
 *  - Threads: one host thread per plan at a time; distinct plans are independent.
 *  - Errors: no exception or abort crosses the ABI.  ttnn_last_error() returns a
 *    thread-local message describing the last non-OK status.
 */
#ifndef TTNN_H
#define TTNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TTNN_MAX_ORDER 8
#define TTNN_MAX_NODES 64

typedef struct ttnn_plan_s* ttnn_plan_t;

typedef enum {
  TTNN_OK = 0,
  TTNN_E_INVALID = -1,  /* bad argument (null pointer, size, enum value)           */
  TTNN_E_TREE = -2,     /* the index tree violates Def. 3 as read by this library   */
  TTNN_E_RANGE = -3,    /* an update box or node id lies outside the tensor / tree  */
  TTNN_E_NOMEM = -4,    /* device allocation failed                                */
  TTNN_E_HIP = -5,      /* a HIP runtime call failed (sticky)                      */
  TTNN_E_STATE = -6,    /* call out of order (e.g. reconstruct before assemble)    */
  TTNN_E_NUMERIC = -7   /* non-finite sketch, or a node whose Omega has rank 0     */
} ttnn_status;

/* TTNN_KR: the TTNN sketches of Sec. 4 with the Khatri-Rao structured maps of Sec. 7,
 * for tensors given in TTN format (rounding / recompression, e.g. of sums of TTNs): see
 * ttnn_sketch_update_ttn. */
typedef enum { TTNN_TTNN = 0, TTNN_STTNN = 1, TTNN_KR = 2 } ttnn_variant;

/* Per-mode factors of TTNN_KR plans are seeded with map tags 2 (TTNN_KR_TAG_BASE + mu)
 * + kind (mu 0-based), after the per-node tags 2 v + kind of the dense maps. */
#define TTNN_KR_TAG_BASE 64

/* Storage / multiply precision of the tensor, of the DRM copies read by the hot
 * kernels and of the MFMA inputs.  Accumulators and the whole recovery phase are
 * FP64 regardless. */
typedef enum { TTNN_F64 = 0, TTNN_F32 = 1, TTNN_BF16 = 2 } ttnn_dtype;

/* Sketch kinds readable through ttnn_read_sketch (all FP64, column-major):
 *   R      right sketch R_t = T^{t} X_t (STTNN: on the contracted tensor), n_t x r_t
 *   OMEGA  intersection sketch Omega_t = Y_t^T R_t, (r_t + p_t) x r_t
 *   PSI    leaf: R_t; internal: (Y_cm^T kron ... kron Y_c1^T) R_t, prod(r_c+p_c) x r_t
 *          (child c1 is the fastest index); root: T contracted with Y_c^T over every
 *          child, prod(r_c + p_c) x 1 */
typedef enum { TTNN_SK_R = 0, TTNN_SK_OMEGA = 1, TTNN_SK_PSI = 2 } ttnn_sketch_kind;

/* The problem of Sec. 4 / Alg. 2 plus the DRM seed and the precision.
 * Tree: node i has parent parent[i] (-1 for exactly one node, the root) and covers
 * the contiguous 0-based mode interval [first_mode[i], last_mode[i]].  The root
 * covers [0, order-1]; the children of a node are disjoint intervals inside its own
 * (Def. 3: a node contains the union of its children), ordered by first mode.  Modes
 * of a node in none of its children are its free modes: each acts as a child whose
 * maps, projector and core are identities (the paper's convention for dummy nodes),
 * so its index appears in the node's core at its mode position with size n_mu; the
 * tensor-train chain of the paper's Fig. 4 is {1..d} > {1..d-1} > .. > {1}.  Free modes
 * have no ids, DRMs, sketches or cores of their own (ttnn_reuse_set lists nodes only);
 * TTNN_KR plans and ttnn_ttn_dot take trees without them.
 * rank[i] = r_t >= 1 and oversample[i] = p_t >= 0 for non-root nodes (ignored at
 * the root), with r_t <= 64, r_t + p_t <= 256, and the recovery of the node within one
 * workgroup's LDS, 2 (r_t + p_t, rounded up to odd) r_t doubles next to 4 KB of its
 * own: every r_t + p_t <= 256 for r_t <= 38, p_t <= 159 at r_t = 48, p_t <= 91 at
 * r_t = 64 (TTNN_E_INVALID otherwise).  eps_factor: the pseudo-inverse keeps singular values of R_t above
 * eps_factor * ||R_t||_2; 0 selects 10 * 2^-52, which suits FP64 sketches.  With FP32
 * sketches a threshold at the FP32 noise level (about 10 * 2^-23) drops the directions
 * that noise creates and gives markedly smaller errors at ranks where the tensor's
 * spectrum has fallen below it.
 * visit: NULL for the lexicographic order of the STTNN sketches (Sec. 5: level by
 * level, the children of each node left to right), else an array of num_nodes entries
 * where visit[i] is the place of node i among its siblings in the order they are
 * visited (0 = first; the root's entry is ignored): a permutation of 0..m-1 over the
 * m children of every node.  Sec. 5 leaves the order free; node t then reuses the
 * contractions of S_t = the siblings of t visited before it together with those of
 * every ancestor of t, so the order changes the shapes of the X_t (their rows run over
 * the indices of T_{S_t} outside I_t) and the cost of the sketch phase, not the form of
 * the approximant.  ttnn_order_search picks one.  TTNN and TTNN_KR plans check the
 * array and ignore it.  The one-pass kernels of STTNN serve the lexicographic order;
 * other orders take the generic contractions. */
typedef struct {
  int32_t order;
  const int64_t* dims;
  int32_t num_nodes;
  const int32_t* parent;
  const int32_t* first_mode;
  const int32_t* last_mode;
  const int32_t* rank;
  const int32_t* oversample;
  int32_t variant;   /* ttnn_variant */
  int32_t dtype;     /* ttnn_dtype   */
  uint64_t seed;
  double eps_factor;
  const int32_t* visit;
} ttnn_problem;

/* Validate the problem, allocate the plan's device memory, and generate every DRM
 * on `stream`: X_t (m_t x r_t) and Y_t (n_t x (r_t + p_t)) with i.i.d. N(0,1) entries
 * (Sec. 4, eq. "sketch"; Gaussian maps as assumed by Lemma 4 and Theorem 2).  Entry
 * (row, col) of map kind (0 = X, 1 = Y) of level-order node v is Box-Muller applied
 * to Philox4x32-10 (Salmon et al., SC'11) with counter (lo32 row, hi32 row, col,
 * 2 v + kind) and key (lo32 seed, hi32 seed), using the 53 high bits of each 64-bit
 * half as u1 = (a + 1) 2^-53 and u2 = b 2^-53, and fixed-order binary64 series for
 * ln and cos(2 pi .) so that the FP64 value is reproducible bit for bit; the FP32
 * copy is its round-to-nearest value and the BF16 copy the round-to-nearest-even of
 * the FP32 bits.  An F32 / BF16 plan uses its rounded copy for every use of a map
 * (the sweeps, the FP64 intermediates and epilogue, rank-1 updates): its FP64 array
 * holds the rounded values exactly, so that each node has one X_t and one Y_t and the
 * projector identities of Sec. 4 / Sec. 5 hold for the sketches it computes.  Rows of
 * X_t run column-major over the modes outside I_t (TTNN) or over the indices of the
 * contracted tensor outside I_t (STTNN, contracted groups kept in place); rows of Y_t
 * run column-major over I_t.  Accumulators start at 0. */
ttnn_status ttnn_plan_create(const ttnn_problem* problem, void* stream, ttnn_plan_t* out);
/* A TTNN_KR plan (dtype F64, one rank r and one oversample p for every node) draws
 * instead, for every mode mu, the factors X_mu (n_mu x r) and Y_mu (n_mu x (r + p)) of
 * Sec. 7 with tags 2 (TTNN_KR_TAG_BASE + mu) + kind, row-major, by the same generator.
 * Its maps are X_t = khatri-rao of X_mu over the modes outside I_t and Y_t =
 * khatri-rao of Y_mu over I_t, never formed: column j of each is the Kronecker product
 * of the factors' columns j, entry (i_1, .., i_d) of it prod_mu X_mu(i_mu, j), rows
 * column-major as for the dense maps.  It keeps Omega_t, Psi_t (R_t for leaves) and the
 * root Psi as accumulators, takes TTN-format updates only (ttnn_sketch_update_ttn), and
 * its recovery is that of every plan.  It sizes the dense reconstruction only when its
 * intermediates stay below 2^27 doubles (else ttnn_reconstruct returns TTNN_E_STATE). */

/* STTNN visiting orders (Sec. 5 leaves the order of the nodes free and calls the best
 * one a combinatorial problem).  Cost model of one whole-tensor sketch pass:
 *   TTNN_COST_FLOPS  2 x (entries of the operand) x (columns of the map) summed over
 *                    every R_t = (T_{S_t})^{t} X_t and every step of the chains of
 *                    contractions T x_s Y_s^T that the S_t and the root sketch need
 *                    (each once; identity maps of free modes cost nothing);
 *   TTNN_COST_MAPS   entries of every X_t (the maps the sweep streams).
 * The cost of a subtree is the product of k_s / n_s over the groups contracted before
 * it times its cost with nothing contracted, so the order of each node's children can
 * be chosen on its own, deepest nodes first.
 * ttnn_order_cost: the cost of problem->visit (NULL: lexicographic).
 * ttnn_order_search: writes to visit (num_nodes entries, host memory) the order of
 * least cost, a valid problem->visit, and its cost to *cost: exhaustive over the
 * orders of the children of every node, so the optimum of the model; ties keep the
 * lexicographic order.  Host-only: nothing is allocated or launched.  Both take STTNN
 * problems only (TTNN_E_INVALID otherwise) and validate them like ttnn_plan_create. */
typedef enum { TTNN_COST_FLOPS = 0, TTNN_COST_MAPS = 1 } ttnn_cost;
ttnn_status ttnn_order_cost(const ttnn_problem* problem, int32_t objective, double* cost);
ttnn_status ttnn_order_search(const ttnn_problem* problem, int32_t objective, int32_t* visit, double* cost);

/* Device bytes a plan for `problem` needs (its DRMs in FP64 and in the compute dtype,
 * FP64 accumulators, cores' scratch and partial sums), computed on the host without
 * allocating or launching anything; 0 if the problem is invalid (ttnn_last_error says
 * why). */
size_t ttnn_workspace_bytes(const ttnn_problem* problem);

/* The plan of ttnn_plan_create, built inside a device workspace the caller owns:
 * d_ws (256-byte aligned) of ws_bytes >= ttnn_workspace_bytes(problem).  Every device
 * array of the plan is a view into d_ws; the DRMs are generated and the accumulators
 * zeroed on `stream`.  The workspace must stay allocated, and be used by nothing else,
 * until ttnn_destroy / ttnn_destroy_async, which never free it.  TTNN_E_INVALID if the
 * workspace is missing, misaligned or too small. */
ttnn_status ttnn_plan(const ttnn_problem* problem, void* d_ws, size_t ws_bytes, void* stream, ttnn_plan_t* out);
ttnn_status ttnn_destroy(ttnn_plan_t plan);

/* Releases the plan without waiting: the device memory of a ttnn_plan_create plan
 * (stream ordered) returns to the device pool when `stream` reaches this call (a
 * caller's workspace stays the caller's), and the handle is invalid on return.  Every piece of work on the plan must be enqueued on `stream`
 * (or ordered before this point on it).  For serving loops that retire streams
 * while other work is in flight. */
ttnn_status ttnn_destroy_async(ttnn_plan_t plan, void* stream);

/* Device bytes owned by the plan (DRMs in FP64 and in the compute dtype, FP64
 * accumulators, cores and scratch).  Used for admission by footprint. */
size_t ttnn_footprint_bytes(ttnn_plan_t plan);

/* The footprint ttnn_plan_create would allocate for `problem`, computed on the host
 * without allocating or launching anything (admission before creation).  Validates
 * the problem like ttnn_plan_create. */
ttnn_status ttnn_footprint_estimate(const ttnn_problem* problem, size_t* bytes);

/* Streaming update (Sec. 4, linearity): add alpha * sketch(H) to the accumulators,
 * where H is zero outside the box [offset, offset + extent) and equals the block
 * d_block (plan dtype) inside it.  strides: NULL for a packed column-major block
 * (extent[0] fastest), else the element stride of each mode (>= 1 on modes of extent
 * > 1), so that box entry (i_1, .., i_d) is d_block[sum_mu i_mu strides[mu]]: a slice
 * of a larger resident array is read in place (e.g. strides = the array's packed
 * strides).  A strided block takes the generic contraction kernels (one of at least
 * 2^22 entries is first copied, in stream order, into a packed block from the library's
 * pool, which gives the same bits faster); packed whole tensors take the one-pass
 * kernels.  The whole tensor is offset = 0, extent = dims.
 * Empty boxes are a no-op. */
ttnn_status ttnn_sketch_update(ttnn_plan_t plan, const void* d_block, const int64_t* offset,
                               const int64_t* extent, const int64_t* strides, double alpha, void* stream);

/* Rank-1 update H = a_1 o a_2 o ... o a_d: d_factors is a host array of `order`
 * device pointers to FP64 vectors of length n_mu. */
ttnn_status ttnn_sketch_update_rank1(ttnn_plan_t plan, const double* const* d_factors,
                                     double alpha, void* stream);

/* nterms rank-1 updates in one call (streaming by linearity, Sec. 4): d_factors is a
 * host array of nterms x order device pointers, term-major (term i's factor of mode mu
 * at d_factors[i * order + mu]), alphas a host array of nterms scales.  Bitwise equal
 * to nterms calls of ttnn_sketch_update_rank1 in order; up to 16 terms share one read
 * of each map (a rank-1 update reads every map once, so a batch of terms costs about
 * one term's map traffic; see ttnn_set_rank1_form).  nterms = 0 is a no-op. */
ttnn_status ttnn_sketch_update_rank1_batched(ttnn_plan_t plan, int32_t nterms, const double* const* d_factors,
                                             const double* alphas, void* stream);

/* How the plan's rank-1 updates form X_t^T v_t (Sec. 4 linearity; the same sums, in
 * FP64 products, in a different association):
 *   TTNN_R1_TERMWISE (default)  a GEMV per term over the map's rows, fastest for terms
 *                               applied one or two at a time;
 *   TTNN_R1_GROUPED             where a map has two fastest factor positions of 16..64
 *                               and 4..64 values, at most 48 columns, a block of the
 *                               first position's rows within 6 KB and at least 256
 *                               workgroups' work (blocks, each split over up to an
 *                               eighth of the second position's length in workgroups
 *                               where there are fewer than 1,024 blocks),
 *                               the two positions are contracted on the FP64
 *                               MFMA for up to 16 terms at once: in groups of 16 a term
 *                               costs about a quarter of a term-wise one in the same
 *                               group and an eighth of a lone term, alone 1.3 times a
 *                               lone term; other maps keep the per-term form.
 * Every rank-1 update of a plan takes its plan's form, so a term's result is bitwise
 * the same in any batch; the two forms agree to FP64 rounding.  Set it before the
 * plan's first rank-1 update.  TTNN_E_INVALID for another value. */
typedef enum { TTNN_R1_TERMWISE = 0, TTNN_R1_GROUPED = 1 } ttnn_rank1_form;
ttnn_status ttnn_set_rank1_form(ttnn_plan_t plan, int32_t form);

/* Several box updates, possibly for different plans, in one call (continuous
 * batching of streamed updates, Sec. 4 linearity).  The call works in rounds: a
 * round takes the earliest remaining update of every plan; the box updates of a
 * round whose plans share tree shape, variant and dtype (sizes and boxes may differ)
 * run each step of the generic path as one launch over all of them (descriptor
 * tables staged through pinned memory); whole-tensor updates run alone.  For every
 * plan the result is bitwise the result of applying its updates one by one with
 * ttnn_sketch_update: each update's arithmetic and reduction order depend only on its
 * own box.  All descriptors are validated before anything is enqueued. */
typedef struct {
  ttnn_plan_t plan;
  const void* d_block;
  int64_t offset[TTNN_MAX_ORDER];
  int64_t extent[TTNN_MAX_ORDER];
  int64_t strides[TTNN_MAX_ORDER];   /* strides[0] == 0: packed; else as in ttnn_sketch_update */
  double alpha;
} ttnn_update_desc;
ttnn_status ttnn_sketch_update_batched(int32_t n, const ttnn_update_desc* descs, void* stream);

/* TTN-format update of a TTNN_KR plan (Sec. 7; Sec. 4 linearity): add alpha * the
 * sketches of the tensor with TTN cores d_cores[c] (device pointers by caller node id,
 * the core layout of ttnn_assemble: leaf (n_t, s_t), internal (s_c1, .., s_cm, s_t),
 * root (s_c1, .., s_cm), column-major FP64) and ranks s_t = ranks[c] in [1, 4096] (the
 * root's ignored).  Computed by contracting the tree, at a cost linear in the mode
 * sizes and without forming the tensor:
 *   dx_t, dy_t = the subtree of t contracted with the X (Y) columns j of its modes,
 *   u_t = everything outside the subtree of t contracted with the X columns j,
 *   Omega_t += alpha dy_t^T u_t,  leaf R_t = Psi_t += alpha U_t u_t,
 *   internal Psi_t += alpha B_t x_c dy_c^T (each child) x_t u_t^T,
 *   root Psi_0 += alpha B_0 x_c dy_c^T (each child).
 * d_work: device scratch of ttnn_update_ttn_work_bytes bytes (256-byte aligned), or
 * NULL to take it from the library's per-device pool for the call (stream ordered).
 * TTNN_E_STATE on other plans; ttnn_sketch_update / _rank1 / _batched return
 * TTNN_E_STATE on TTNN_KR plans. */
ttnn_status ttnn_update_ttn_work_bytes(ttnn_plan_t plan, const int32_t* ranks, size_t* bytes);
ttnn_status ttnn_sketch_update_ttn(ttnn_plan_t plan, const double* const* d_cores, const int32_t* ranks,
                                   double alpha, void* d_work, size_t work_bytes, void* stream);

/* Inner product <A, B> of two tensors in TTN format on the plan's tree (any plan;
 * cores and ranks as for ttnn_sketch_update_ttn), by Gram matrices of the subtrees,
 * deepest first: G_leaf = U_a^T U_b, G_t = B_a x_c G_c (each child) contracted with
 * B_b.  The result goes to d_out[0] (device memory) in stream order.  Errors of a
 * rounding follow as ||A - B||^2 = <A,A> - 2 <A,B> + <B,B>, which resolves relative
 * errors down to about 1e-7 in FP64.  d_work as for ttnn_sketch_update_ttn, sized by
 * ttnn_ttn_dot_work_bytes. */
ttnn_status ttnn_ttn_dot_work_bytes(ttnn_plan_t plan, const int32_t* ranks_a, const int32_t* ranks_b, size_t* bytes);
ttnn_status ttnn_ttn_dot(ttnn_plan_t plan, const double* const* d_a, const int32_t* ranks_a, const double* const* d_b,
                         const int32_t* ranks_b, double* d_out, void* d_work, size_t work_bytes, void* stream);

/* Per-mode factor of a TTNN_KR plan: kind 0 = X_mu (n_mu x r), 1 = Y_mu (n_mu x (r + p)),
 * row-major FP64, copied to d_out. */
ttnn_status ttnn_read_factor(ttnn_plan_t plan, int32_t mode, int32_t kind, double* d_out, void* stream);

/* Shape of node `node`'s core (column-major, parent rank index last):
 *   leaf (n_t, r_t); internal (r_c1, ..., r_cm, r_t); root (r_c1, ..., r_cm), with n_mu
 *   in place of r_c at the position of a free mode mu. */
ttnn_status ttnn_core_shape(ttnn_plan_t plan, int32_t node, int32_t* ndim, int64_t* shape);

/* Recovery phase (Sec. 4, Alg. 2; internal nodes at every level >= 1):
 *   [Q_t, Rt_t] = qr(Omega_t) with diag(Rt_t) >= 0;  Rt_t^{+eps} by one-sided Jacobi SVD;
 *   leaf B_t = Psi_t Rt_t^{+eps}; internal B_t = (kron Q_c^T) Psi_t Rt_t^{+eps};
 *   root B_0 = (kron Q_c^T) Psi_0.
 * All in FP64 on the GPU.  d_cores: host array of num_nodes device pointers (caller
 * node ids), each with room for prod(core shape) doubles.  Returns TTNN_E_NUMERIC
 * (after writing the cores) if a sketch was not finite or a node's Omega has numerical
 * rank 0 (its pseudo-inverse, and so its contribution, is zero: the zero tensor gives
 * finite cores that reconstruct it exactly); the flag is read back synchronously, so
 * this call synchronises `stream`. */
ttnn_status ttnn_assemble(ttnn_plan_t plan, double* const* d_cores, void* stream);

/* The same recovery phase, enqueued on `stream` without waiting: returns TTNN_OK
 * once the work is enqueued (TTNN_E_INVALID for bad arguments).  The cores are valid
 * when `stream` reaches the end of this work.  The numerical status (non-finite
 * sketch, or a node whose Omega has numerical rank 0) is or-ed into the plan's
 * sticky status, which ttnn_assemble_status reports.  For serving loops that
 * assemble on demand without draining the stream. */
ttnn_status ttnn_assemble_async(ttnn_plan_t plan, double* const* d_cores, void* stream);

/* TTNN_E_NUMERIC if any ttnn_assemble / ttnn_assemble_async of this plan since the
 * previous call found a non-finite sketch or a rank-0 node, else TTNN_OK; clears the
 * sticky status.  Synchronises `stream` (use the stream the assemblies ran on). */
ttnn_status ttnn_assemble_status(ttnn_plan_t plan, void* stream);

/* The same query without waiting: enqueues on `stream` a copy of the sticky status
 * (0 = sound, 1 = TTNN_E_NUMERIC) into *h_status, which must be pinned host memory
 * (hipHostMalloc) that the caller owns, and clears it.  *h_status is valid once
 * `stream` has passed the call (e.g. an event recorded after it has completed). */
ttnn_status ttnn_assemble_status_async(ttnn_plan_t plan, int32_t* h_status, void* stream);

/* Dense reconstruction (Def. 5, matricised form) from cores laid out as written by
 * ttnn_assemble: d_out receives prod(dims) values of dtype out_dtype, column-major. */
ttnn_status ttnn_reconstruct(ttnn_plan_t plan, const double* const* d_cores, void* d_out,
                             int32_t out_dtype, void* stream);

/* Squared Frobenius norms ||a - b||^2 and ||b||^2 of two dense arrays of n entries,
 * a of dtype a_dtype, b FP64 (error of a reconstruction).  Deterministic; synchronises
 * `stream` and writes h_out[0..1].  Its 16 KB of partial sums come from the library's
 * per-device pool, stream ordered. */
ttnn_status ttnn_diff_norms(const void* d_a, int32_t a_dtype, const double* d_b, int64_t n,
                            double* h_out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): ttnn_diff_norms with its partial
 * sums in a library-static device array (2 x 1024 doubles per device, 16 KB, the same
 * for every n >= 0) instead of a fresh allocation, and without a host
 * synchronisation: the two sums ||a - b||^2 and ||b||^2 go to d_out[0..1] (device
 * memory) in stream order, bitwise equal to ttnn_diff_norms's.  Calls that overlap on
 * one device (other streams or threads) share that array and race. */
ttnn_status ttnn_diff_norms_noalloc(const void* d_a, int32_t a_dtype, const double* d_b, int64_t n, double* d_out,
                                    void* stream);

/* Parity hooks. */
ttnn_status ttnn_sketch_shape(ttnn_plan_t plan, int32_t node, int32_t kind, int64_t* rows,
                              int64_t* cols);
ttnn_status ttnn_read_sketch(ttnn_plan_t plan, int32_t node, int32_t kind, double* d_out,
                             void* stream);
/* DRM of node `node` (kind 0 = X, 1 = Y) as stored for `dtype` (the FP64 array, or the
 * FP32 / BF16 copy of an F32 / BF16 plan, whose values the FP64 array then holds),
 * row-major rows x cols; BF16 as uint16. */
ttnn_status ttnn_drm_shape(ttnn_plan_t plan, int32_t node, int32_t kind, int64_t* rows,
                           int64_t* cols);
ttnn_status ttnn_read_drm(ttnn_plan_t plan, int32_t node, int32_t kind, int32_t dtype,
                          void* d_out, void* stream);

/* Canonical (level-order) id of caller node `node`, and the STTNN reuse set S_t
 * (Sec. 5, Fig. 5) as caller ids (ids: room for num_nodes), in the order its chain of
 * contractions takes them: the groups of the ancestors' levels first, from the top
 * down, each level in visiting order (left to right for the lexicographic order). */
ttnn_status ttnn_level_id(ttnn_plan_t plan, int32_t node, int32_t* level_id);
ttnn_status ttnn_reuse_set(ttnn_plan_t plan, int32_t node, int32_t* count, int32_t* ids);

/* Measurement hook.  With timing on, every update records two HIP events on its
 * stream: before its first kernel and after its sweep, the kernel that streams the
 * tensor (the one-pass fused kernel where it applies; otherwise the whole update).
 * ttnn_sweep_time_ms waits for the second event of the last update and returns the
 * elapsed milliseconds (TTNN_E_STATE if no update was timed).  Off by default; it
 * adds no synchronisation to the update itself. */
ttnn_status ttnn_set_timing(ttnn_plan_t plan, int32_t on);
ttnn_status ttnn_sweep_time_ms(ttnn_plan_t plan, float* ms);
/* What the timed sweep of a whole-tensor update computes, for accounting its work:
 * 0 the whole update (no one-pass kernel applies); 1 one-pass STTNN kernel (R_A, Z_A,
 * R_1, R_2 = Z1 X_2 in the kernel); 2 one-pass STTNN kernel writing Z1 out (R_2 formed
 * after it by a streaming contraction); 3 one-pass TTNN-mode kernel (R_A, Z_A, R_1,
 * R_B). */
ttnn_status ttnn_sweep_kind(ttnn_plan_t plan, int32_t* kind);

/* Host-side sizing hooks (pure arithmetic, no device; for tests and tools).
 * ttnn_right_sketch_split: how a whole-tensor right sketch R = T^{t} X_t on the MFMA
 * form is split over its contraction: the operand is [contraction_run][rows][runs]
 * (the contraction runs over contraction_run x runs values, rows = n_t), r columns;
 * nchunks chunks of kchunk values, each writing a rows x r FP64 partial into scratch of
 * scratch_elems doubles (nchunks * rows * r <= scratch_elems).  TTNN_E_INVALID if the
 * shape is not covered or the scratch cannot hold one chunk.
 * ttnn_chain_head_split: the first contraction of an STTNN / root chain, Y_g^T applied
 * to the raw tensor for a group g at mode 1 (group_rows = n_g contracted values per
 * row, `rows` output rows of k values): *in_place = 1 when the partial scratch cannot
 * hold two chunks, the single chunk then being written straight into the chain buffer
 * of rows * k values; otherwise the split through the scratch. */
ttnn_status ttnn_right_sketch_split(int64_t contraction_run, int64_t rows, int64_t runs, int32_t r, int32_t dtype,
                                    size_t scratch_elems, int32_t compute_units, int64_t* nchunks, int64_t* kchunk);
ttnn_status ttnn_chain_head_split(int64_t group_rows, int64_t rows, int32_t k, int32_t dtype, size_t scratch_elems,
                                  int32_t compute_units, int32_t* in_place, int64_t* nchunks, int64_t* kchunk);

/* Zero the accumulators and clear a sticky error. */
ttnn_status ttnn_reset(ttnn_plan_t plan, void* stream);

const char* ttnn_status_string(ttnn_status s);
const char* ttnn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TTNN_H */
