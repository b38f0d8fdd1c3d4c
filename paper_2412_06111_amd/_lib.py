"""ctypes binding of libttnn.so (argument marshalling only).

Every computation happens in the library's HIP kernels; PyTorch is used for
device memory and streams.  Importing this module fails loudly when the library
has not been built.
"""

import ctypes as C
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libttnn.so")

F64, F32, BF16 = 0, 1, 2
TTNN, STTNN, KR = 0, 1, 2
SK_R, SK_OMEGA, SK_PSI = 0, 1, 2
MAX_ORDER = 8

TORCH_DTYPE = {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16}
DTYPE_NAME = {F64: "f64", F32: "f32", BF16: "bf16"}
DTYPE_OF_NAME = {"f64": F64, "f32": F32, "bf16": BF16}
VARIANT_OF_NAME = {"ttnn": TTNN, "sttnn": STTNN, "kr": KR}


class TTNNError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ttnn status {status}: {msg}")
        self.status = status


class Problem(C.Structure):
    _fields_ = [
        ("order", C.c_int32), ("dims", C.POINTER(C.c_int64)),
        ("num_nodes", C.c_int32), ("parent", C.POINTER(C.c_int32)),
        ("first_mode", C.POINTER(C.c_int32)), ("last_mode", C.POINTER(C.c_int32)),
        ("rank", C.POINTER(C.c_int32)), ("oversample", C.POINTER(C.c_int32)),
        ("variant", C.c_int32), ("dtype", C.c_int32), ("seed", C.c_uint64), ("eps_factor", C.c_double),
        ("visit", C.POINTER(C.c_int32)),
    ]


class UpdateDesc(C.Structure):
    _fields_ = [
        ("plan", C.c_void_p), ("d_block", C.c_void_p),
        ("offset", C.c_int64 * MAX_ORDER), ("extent", C.c_int64 * MAX_ORDER), ("strides", C.c_int64 * MAX_ORDER),
        ("alpha", C.c_double),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2412_06111_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P64 = C.POINTER(i64)
    P32 = C.POINTER(i32)
    PSZ = C.POINTER(C.c_size_t)
    sigs = {
        "ttnn_update_ttn_work_bytes": [vp, P32, PSZ],
        "ttnn_sketch_update_ttn": [vp, C.POINTER(vp), P32, dbl, vp, C.c_size_t, vp],
        "ttnn_ttn_dot_work_bytes": [vp, P32, P32, PSZ],
        "ttnn_ttn_dot": [vp, C.POINTER(vp), P32, C.POINTER(vp), P32, vp, vp, C.c_size_t, vp],
        "ttnn_read_factor": [vp, i32, i32, vp, vp],
        "ttnn_plan_create": [C.POINTER(Problem), vp, C.POINTER(vp)],
        "ttnn_plan": [C.POINTER(Problem), vp, C.c_size_t, vp, C.POINTER(vp)],
        "ttnn_destroy": [vp],
        "ttnn_destroy_async": [vp, vp],
        "ttnn_sketch_update": [vp, vp, P64, P64, P64, dbl, vp],
        "ttnn_sketch_update_rank1": [vp, C.POINTER(vp), dbl, vp],
        "ttnn_sketch_update_rank1_batched": [vp, i32, C.POINTER(vp), C.POINTER(dbl), vp],
        "ttnn_sketch_update_batched": [i32, C.POINTER(UpdateDesc), vp],
        "ttnn_core_shape": [vp, i32, C.POINTER(i32), P64],
        "ttnn_assemble": [vp, C.POINTER(vp), vp],
        "ttnn_assemble_async": [vp, C.POINTER(vp), vp],
        "ttnn_assemble_status": [vp, vp],
        "ttnn_assemble_status_async": [vp, vp, vp],
        "ttnn_sweep_kind": [vp, C.POINTER(i32)],
        "ttnn_reconstruct": [vp, C.POINTER(vp), vp, i32, vp],
        "ttnn_diff_norms": [vp, i32, vp, i64, C.POINTER(dbl), vp],
        "ttnn_sketch_shape": [vp, i32, i32, P64, P64],
        "ttnn_read_sketch": [vp, i32, i32, vp, vp],
        "ttnn_drm_shape": [vp, i32, i32, P64, P64],
        "ttnn_read_drm": [vp, i32, i32, i32, vp, vp],
        "ttnn_level_id": [vp, i32, C.POINTER(i32)],
        "ttnn_reuse_set": [vp, i32, C.POINTER(i32), C.POINTER(i32)],
        "ttnn_reset": [vp, vp],
        "ttnn_set_timing": [vp, i32],
        "ttnn_set_rank1_form": [vp, i32],
        "ttnn_footprint_estimate": [C.POINTER(Problem), C.POINTER(C.c_size_t)],
        "ttnn_order_cost": [C.POINTER(Problem), i32, C.POINTER(dbl)],
        "ttnn_order_search": [C.POINTER(Problem), i32, P32, C.POINTER(dbl)],
        "ttnn_sweep_time_ms": [vp, C.POINTER(C.c_float)],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.ttnn_footprint_bytes.argtypes = [vp]
    lib.ttnn_footprint_bytes.restype = C.c_size_t
    lib.ttnn_workspace_bytes.argtypes = [C.POINTER(Problem)]
    lib.ttnn_workspace_bytes.restype = C.c_size_t
    lib.ttnn_status_string.argtypes = [C.c_int]
    lib.ttnn_status_string.restype = C.c_char_p
    lib.ttnn_last_error.argtypes = []
    lib.ttnn_last_error.restype = C.c_char_p
    return lib


lib = _load()


def check(status):
    if status != 0:
        raise TTNNError(status, (lib.ttnn_last_error() or b"").decode())


def check_block(block, dtype, extent, d, strides=None):
    """Argument checks of a box update's block (raised, not asserted, so they hold under
    python -O).  `dtype` is the plan's torch dtype, `extent` the box, `d` the tensor
    order.  Without strides the block must be contiguous with exactly prod(extent)
    entries; with strides (elements, one per mode) it must hold every addressed entry."""
    if not isinstance(block, torch.Tensor):
        raise TypeError(f"block must be a torch.Tensor, got {type(block).__name__}")
    if block.dtype != dtype:
        raise TypeError(f"block dtype {block.dtype} differs from the plan dtype {dtype}")
    if len(extent) != d:
        raise ValueError(f"extent has {len(extent)} modes, the tensor has {d}")
    n = 1
    for e in extent:
        if int(e) < 0:
            raise ValueError(f"negative extent {tuple(extent)}")
        n *= int(e)
    if strides is None:
        if not block.is_contiguous():
            raise ValueError("block must be contiguous (column-major box, extent[0] fastest); pass strides "
                             "for a strided view")
        if block.numel() != n:
            raise ValueError(f"block has {block.numel()} entries, the box {tuple(extent)} has {n}")
    else:
        if len(strides) != d:
            raise ValueError(f"strides has {len(strides)} modes, the tensor has {d}")
        if n > 0:
            last = sum((int(e) - 1) * int(s) for e, s in zip(extent, strides))
            room = block.untyped_storage().nbytes() // block.element_size() - block.storage_offset()
            if any(int(s) < 0 for s in strides) or last >= room:
                raise ValueError(f"strides {tuple(strides)} address entries outside the block's storage")
    if not block.is_cuda:
        raise TypeError("block must be a CUDA (HIP) tensor")


class _nullctx:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False


def stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------- trees
def _modes(spec):
    if isinstance(spec, int):
        return (abs(spec),)
    if isinstance(spec, frozenset):
        return tuple(sorted(spec))
    out = ()
    for c in spec:
        out += _modes(c)
    return out


def tree_arrays(spec):
    """Nested-tuple tree (1-based modes) -> caller arrays in depth-first order.
    A negative int -m inside a tuple is a free mode m of that node (no node of its
    own: the node's interval covers it, no child does).
    Returns (parent, first, last, modes_of_node)."""
    parent, first, last, modes = [], [], [], []

    def walk(s, par):
        m = _modes(s)
        me = len(parent)
        parent.append(par)
        first.append(m[0] - 1)
        last.append(m[-1] - 1)
        modes.append(m)
        if isinstance(s, tuple):
            for c in s:
                if not (isinstance(c, int) and c < 0):
                    walk(c, me)

    walk(spec, -1)
    return parent, first, last, modes


def _visit_lists(spec):
    """{modes of an internal node: [modes of its children in the listed order]}."""
    out = {}

    def walk(s):
        if not isinstance(s, tuple):
            return
        kids = [c for c in s if not (isinstance(c, int) and c < 0)]
        out[tuple(sorted(_modes(s)))] = [tuple(sorted(_modes(c))) for c in kids]
        for c in kids:
            walk(c)

    walk(spec)
    return out


def visit_places(spec, visit):
    """The caller arrays' `visit` entries of a visiting order given as a spec of the same
    tree with each node's children listed in the order they are visited."""
    par, _, _, modes = tree_arrays(spec)
    lists = _visit_lists(visit)
    out = []
    for i, p in enumerate(par):
        if p < 0:
            out.append(0)
            continue
        sib = lists.get(tuple(sorted(modes[p])))
        me = tuple(sorted(modes[i]))
        if sib is None or me not in sib:
            raise ValueError(f"the visiting order does not list node {modes[i]} under {modes[p]}")
        out.append(sib.index(me))
    return out


def visit_spec(spec, places):
    """Inverse of visit_places: the tree spec with each node's children listed in the
    visiting order (free modes after them)."""
    it = iter(range(len(places)))

    def walk(s):
        me = next(it)
        if not isinstance(s, tuple):
            return me, s
        kids = [walk(c) for c in s if not (isinstance(c, int) and c < 0)]
        free = tuple(c for c in s if isinstance(c, int) and c < 0)
        kids.sort(key=lambda kc: places[kc[0]])
        return me, tuple(c for _, c in kids) + free

    return walk(spec)[1]


def _problem(spec, dims, rank, over, variant, dtype, seed, eps_factor, visit=None):
    """Marshal a problem; returns (Problem, keep-alive arrays, node modes)."""
    dims = tuple(int(n) for n in dims)
    d = len(dims)
    variant = VARIANT_OF_NAME[variant] if isinstance(variant, str) else int(variant)
    dtype = DTYPE_OF_NAME[dtype] if isinstance(dtype, str) else int(dtype)
    par, fst, lst, modes = tree_arrays(spec)
    nn = len(par)
    rk = [int(rank[m] if isinstance(rank, dict) else rank) if i else 0 for i, m in enumerate(modes)]
    ov = [int(over[m] if isinstance(over, dict) else over) if i else 0 for i, m in enumerate(modes)]
    arrays = ((C.c_int64 * d)(*dims), (C.c_int32 * nn)(*par), (C.c_int32 * nn)(*fst),
              (C.c_int32 * nn)(*lst), (C.c_int32 * nn)(*rk), (C.c_int32 * nn)(*ov))
    if visit is not None:
        arrays = arrays + ((C.c_int32 * nn)(*visit_places(spec, visit)),)
    a = arrays
    pr = Problem(d, a[0], nn, a[1], a[2], a[3], a[4], a[5], variant, dtype, C.c_uint64(int(seed)),
                 float(eps_factor), a[6] if visit is not None else None)
    return pr, arrays, modes


COST_OF_NAME = {"flops": 0, "maps": 1}


def order_cost(spec, dims, rank, over, visit=None, objective="flops"):
    """Cost of one whole-tensor STTNN sketch pass in the visiting order `visit` (a spec of
    the tree listing children in visiting order; None: lexicographic): leading-order
    flops, or entries of the X_t maps."""
    pr, _keep, _ = _problem(spec, dims, rank, over, STTNN, F64, 1, 0.0, visit)
    out = C.c_double()
    check(lib.ttnn_order_cost(C.byref(pr), COST_OF_NAME[objective], C.byref(out)))
    return float(out.value)


def order_search(spec, dims, rank, over, objective="flops"):
    """The STTNN visiting order of least cost under the library's model; returns
    (visit spec, cost)."""
    pr, _keep, _ = _problem(spec, dims, rank, over, STTNN, F64, 1, 0.0)
    places = (C.c_int32 * pr.num_nodes)()
    out = C.c_double()
    check(lib.ttnn_order_search(C.byref(pr), COST_OF_NAME[objective], places, C.byref(out)))
    return visit_spec(spec, list(places)), float(out.value)


def footprint_estimate(spec, dims, rank, over, variant="ttnn", dtype="f64", visit=None):
    """Device bytes a plan for this problem would own (host-side sizing, no allocation)."""
    pr, _keep, _ = _problem(spec, dims, rank, over, variant, dtype, 1, 0.0, visit)
    out = C.c_size_t()
    check(lib.ttnn_footprint_estimate(C.byref(pr), C.byref(out)))
    return int(out.value)


def workspace_bytes(spec, dims, rank, over, variant="ttnn", dtype="f64", visit=None):
    """Size of the device workspace ttnn_plan needs for this problem."""
    pr, _keep, _ = _problem(spec, dims, rank, over, variant, dtype, 1, 0.0, visit)
    n = int(lib.ttnn_workspace_bytes(C.byref(pr)))
    if n == 0:
        raise TTNNError(-1, (lib.ttnn_last_error() or b"").decode())
    return n


def view_strides(block, extent, d):
    """Column-major element strides of a block given as a torch view of shape
    (e_d, .., e_1) (the layout of a C-contiguous (n_d, .., n_1) tensor), or None when
    it is packed (contiguous) or flat."""
    if block.dim() == d and tuple(block.shape) == tuple(int(e) for e in reversed(extent)) \
            and not block.is_contiguous():
        return tuple(int(block.stride(d - 1 - mu)) for mu in range(d))
    return None


class Plan:
    """A sketching plan: problem of Sec. 4 / Alg. 2 plus seed and precision.

    Device memory: by default a workspace tensor allocated with torch (ttnn_plan; the
    plan's arrays are views into it); `workspace` passes one of the caller's (a CUDA
    uint8 tensor of at least workspace_bytes(...)); pool=True lets the library take a
    block from its own per-device pool (ttnn_plan_create).  visit: the STTNN visiting
    order as a spec of the same tree listing each node's children in the order they are
    visited (None: lexicographic; order_search finds the cheapest)."""

    def __init__(self, spec, dims, rank, over, variant="ttnn", dtype="f64", seed=1, eps_factor=0.0,
                 stream=None, workspace=None, pool=False, visit=None):
        self.spec, self.dims = spec, tuple(int(n) for n in dims)
        self.d = len(self.dims)
        self.variant = VARIANT_OF_NAME[variant] if isinstance(variant, str) else int(variant)
        self.dtype = DTYPE_OF_NAME[dtype] if isinstance(dtype, str) else int(dtype)
        self.visit = visit
        self.problem, self._arrays, modes = _problem(spec, dims, rank, over, variant, dtype, seed, eps_factor,
                                                     visit)
        self.node_modes = modes
        self.node_of_modes = {m: i for i, m in enumerate(modes)}
        self.num_nodes = len(modes)
        self.handle = C.c_void_p()
        self.workspace = None
        if pool:
            check(lib.ttnn_plan_create(C.byref(self.problem), stream_ptr(stream), C.byref(self.handle)))
            return
        need = int(lib.ttnn_workspace_bytes(C.byref(self.problem)))
        if need == 0:
            raise TTNNError(-1, (lib.ttnn_last_error() or b"").decode())
        if workspace is None:
            with torch.cuda.stream(stream) if stream is not None else _nullctx():
                workspace = torch.empty(need, dtype=torch.uint8, device="cuda")
        if not (isinstance(workspace, torch.Tensor) and workspace.is_cuda and workspace.is_contiguous()):
            raise TypeError("workspace must be a contiguous CUDA tensor")
        if workspace.numel() * workspace.element_size() < need:
            raise ValueError(f"workspace of {workspace.numel() * workspace.element_size()} bytes; the plan needs {need}")
        check(lib.ttnn_plan(C.byref(self.problem), C.c_void_p(workspace.data_ptr()),
                            workspace.numel() * workspace.element_size(), stream_ptr(stream), C.byref(self.handle)))
        self.workspace = workspace

    # ------------------------------------------------------------ lifetime
    def close(self):
        if self.handle:
            lib.ttnn_destroy(self.handle)
            self.handle = C.c_void_p()
        self.workspace = None

    def close_async(self, stream=None):
        """Release without waiting: the memory returns to its pool (the library's, or
        torch's for a workspace tensor) when `stream` (on which all of this plan's work
        ran) reaches this point."""
        if self.handle:
            lib.ttnn_destroy_async(self.handle, stream_ptr(stream))
            self.handle = C.c_void_p()
        if self.workspace is not None:
            if stream is not None:
                self.workspace.record_stream(stream)
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def torch_dtype(self):
        return TORCH_DTYPE[self.dtype]

    def footprint(self):
        return int(lib.ttnn_footprint_bytes(self.handle))

    def node(self, modes):
        return self.node_of_modes[tuple(modes)]

    # ------------------------------------------------------------ sketch phase
    def update(self, block, extent=None, offset=None, alpha=1.0, stream=None, strides=None):
        """block: CUDA tensor of the plan dtype holding the box: packed column-major
        (numel == prod(extent)), or a view of shape (e_d, .., e_1) into a larger tensor,
        read in place with its strides; `strides` (elements, mode 1 first) overrides."""
        extent = self.dims if extent is None else tuple(int(e) for e in extent)
        offset = (0,) * self.d if offset is None else tuple(int(o) for o in offset)
        if strides is None:
            strides = view_strides(block, extent, self.d)
        check_block(block, self.torch_dtype, extent, self.d, strides)
        if len(offset) != self.d:
            raise ValueError(f"offset has {len(offset)} modes, the tensor has {self.d}")
        st = None if strides is None else (C.c_int64 * self.d)(*strides)
        check(lib.ttnn_sketch_update(self.handle, C.c_void_p(block.data_ptr()), (C.c_int64 * self.d)(*offset),
                                     (C.c_int64 * self.d)(*extent), st, float(alpha), stream_ptr(stream)))

    def update_rank1(self, factors, alpha=1.0, stream=None):
        """factors: d CUDA float64 vectors, factor mu of length n_mu (the library reads
        exactly that many doubles from each)."""
        if len(factors) != self.d:
            raise ValueError(f"{len(factors)} factors for a tensor of order {self.d}")
        for f, n in zip(factors, self.dims):
            check_block(f, torch.float64, (n,), 1)
        ptrs = (C.c_void_p * self.d)(*[C.c_void_p(f.data_ptr()) for f in factors])
        check(lib.ttnn_sketch_update_rank1(self.handle, ptrs, float(alpha), stream_ptr(stream)))

    def update_rank1_batched(self, terms, alphas, stream=None):
        """terms: a list of factor lists (each as for update_rank1); alphas: one scale per
        term.  Bitwise equal to the terms applied one by one in order."""
        if len(terms) != len(alphas):
            raise ValueError(f"{len(terms)} terms and {len(alphas)} scales")
        flat = []
        for factors in terms:
            if len(factors) != self.d:
                raise ValueError(f"{len(factors)} factors for a tensor of order {self.d}")
            for f, n in zip(factors, self.dims):
                check_block(f, torch.float64, (n,), 1)
            flat += [C.c_void_p(f.data_ptr()) for f in factors]
        ptrs = (C.c_void_p * max(len(flat), 1))(*flat)
        al = (C.c_double * max(len(alphas), 1))(*[float(a) for a in alphas])
        check(lib.ttnn_sketch_update_rank1_batched(self.handle, len(terms), ptrs, al, stream_ptr(stream)))

    # ------------------------------------------------------------ TTN-format inputs
    def _ranks_list(self, ranks):
        if isinstance(ranks, dict):
            return [int(ranks[m]) if i else 0 for i, m in enumerate(self.node_modes)]
        if isinstance(ranks, int):
            return [int(ranks) if i else 0 for i in range(self.num_nodes)]
        return [int(x) for x in ranks]

    def _ttn_args(self, cores, ranks):
        """Core pointers and ranks of a TTN on this plan's tree, in caller node order.
        cores: a list by caller node id or a dict keyed by node modes (CUDA float64,
        contiguous, the layout of assembled cores); ranks: an int (every non-root node),
        a list by caller node id, or a dict keyed by node modes."""
        nn = self.num_nodes
        if isinstance(cores, dict):
            cores = [cores[m] for m in self.node_modes]
        rk = self._ranks_list(ranks)
        if len(cores) != nn or len(rk) != nn:
            raise ValueError(f"a TTN on this tree has {nn} cores and ranks")
        parent = list(self._arrays[1])
        kids = [[] for _ in range(nn)]
        for i in range(1, nn):
            kids[parent[i]].append(i)
        for i in range(nn):
            if i and rk[i] < 1:
                raise ValueError(f"node {i}: TTN rank {rk[i]} < 1")
            if kids[i]:
                want = 1
                for c in kids[i]:
                    want *= rk[c]
                covered = {m for c in kids[i] for m in self.node_modes[c]}
                for m in self.node_modes[i]:                  # free modes of the node
                    if m not in covered:
                        want *= self.dims[m - 1]
                want *= rk[i] if i else 1
            else:
                want = rk[i]
                for m in self.node_modes[i]:
                    want *= self.dims[m - 1]
            check_block(cores[i], torch.float64, (want,), 1)
        ptrs = (C.c_void_p * nn)(*[C.c_void_p(c.data_ptr()) for c in cores])
        return ptrs, (C.c_int32 * nn)(*rk)

    def core_ranks(self):
        """Ranks r_t of the cores this plan assembles, by caller node id (root 0)."""
        return [int(x) if i else 0 for i, x in enumerate(self._arrays[4])]

    def update_ttn(self, cores, ranks, alpha=1.0, stream=None, work=None):
        """Khatri-Rao plans: accumulators += alpha * sketches of the TTN (cores, ranks);
        work: optional CUDA uint8 scratch tensor (else the library's pool serves the call)."""
        ptrs, rk = self._ttn_args(cores, ranks)
        wp, wb = (None, 0) if work is None else (C.c_void_p(work.data_ptr()), work.numel() * work.element_size())
        check(lib.ttnn_sketch_update_ttn(self.handle, ptrs, rk, float(alpha), wp, wb, stream_ptr(stream)))

    def update_ttn_work_bytes(self, ranks):
        """Device scratch (bytes) of one update_ttn with TTN ranks `ranks`."""
        rk = self._ranks_list(ranks)
        out = C.c_size_t()
        check(lib.ttnn_update_ttn_work_bytes(self.handle, (C.c_int32 * self.num_nodes)(*rk), C.byref(out)))
        return int(out.value)

    def ttn_dot(self, a, ranks_a, b, ranks_b, stream=None):
        """<A, B> of two TTNs on this plan's tree, computed on the GPU (waits for it)."""
        pa, ra = self._ttn_args(a, ranks_a)
        pb, rb = self._ttn_args(b, ranks_b)
        out = torch.empty(1, dtype=torch.float64, device="cuda")
        check(lib.ttnn_ttn_dot(self.handle, pa, ra, pb, rb, C.c_void_p(out.data_ptr()), None, 0, stream_ptr(stream)))
        if stream is not None:
            stream.synchronize()
        return float(out.cpu()[0])

    def read_factor(self, mode, kind, stream=None):
        """Per-mode factor of a Khatri-Rao plan: kind 0 = X (n x r), 1 = Y (n x (r + p)), row-major."""
        cols = self.core_ranks()[1] + (0 if kind == 0 else int(self._arrays[5][1]))
        out = torch.empty((self.dims[mode], cols), dtype=torch.float64, device="cuda")
        check(lib.ttnn_read_factor(self.handle, int(mode), int(kind), C.c_void_p(out.data_ptr()), stream_ptr(stream)))
        return out

    def reset(self, stream=None):
        check(lib.ttnn_reset(self.handle, stream_ptr(stream)))

    def set_timing(self, on=True):
        check(lib.ttnn_set_timing(self.handle, 1 if on else 0))

    def set_rank1_form(self, form):
        """"termwise" (default: a GEMV per term) or "grouped" (term groups on the FP64
        MFMA where the maps allow it; for callers that batch rank-1 terms)."""
        check(lib.ttnn_set_rank1_form(self.handle, {"termwise": 0, "grouped": 1}[form]))

    def sweep_kind(self):
        """0 whole update, 1 STTNN one-pass kernel, 2 STTNN one-pass kernel writing Z1
        out, 3 TTNN-mode one-pass kernel (see ttnn_sweep_kind)."""
        k = C.c_int32()
        check(lib.ttnn_sweep_kind(self.handle, C.byref(k)))
        return k.value

    def sweep_time_ms(self):
        """Elapsed time of the last update's sweep kernel (waits for it)."""
        ms = C.c_float()
        check(lib.ttnn_sweep_time_ms(self.handle, C.byref(ms)))
        return ms.value

    # ------------------------------------------------------------ readbacks
    def sketch_shape(self, node, kind):
        r, c = C.c_int64(), C.c_int64()
        check(lib.ttnn_sketch_shape(self.handle, node, kind, C.byref(r), C.byref(c)))
        return r.value, c.value

    def read_sketch(self, node, kind, stream=None):
        r, c = self.sketch_shape(node, kind)
        out = torch.empty(r * c, dtype=torch.float64, device="cuda")
        check(lib.ttnn_read_sketch(self.handle, node, kind, C.c_void_p(out.data_ptr()), stream_ptr(stream)))
        return out.view(c, r).t()        # column-major (r x c)

    def drm_shape(self, node, kind):
        r, c = C.c_int64(), C.c_int64()
        check(lib.ttnn_drm_shape(self.handle, node, kind, C.byref(r), C.byref(c)))
        return r.value, c.value

    def read_drm(self, node, kind, dtype=F64, stream=None):
        r, c = self.drm_shape(node, kind)
        tdt = {F64: torch.float64, F32: torch.float32, BF16: torch.int16}[dtype]
        out = torch.empty((r, c), dtype=tdt, device="cuda")
        check(lib.ttnn_read_drm(self.handle, node, kind, dtype, C.c_void_p(out.data_ptr()), stream_ptr(stream)))
        return out

    def level_id(self, node):
        v = C.c_int32()
        check(lib.ttnn_level_id(self.handle, node, C.byref(v)))
        return v.value

    def reuse_set(self, node):
        cnt = C.c_int32()
        ids = (C.c_int32 * 64)()
        check(lib.ttnn_reuse_set(self.handle, node, C.byref(cnt), ids))
        return [ids[i] for i in range(cnt.value)]

    def core_shape(self, node):
        nd = C.c_int32()
        shp = (C.c_int64 * 16)()
        check(lib.ttnn_core_shape(self.handle, node, C.byref(nd), shp))
        return tuple(shp[i] for i in range(nd.value))

    # ------------------------------------------------------------ recovery
    def alloc_cores(self):
        cores = []
        for i in range(self.num_nodes):
            n = 1
            for s in self.core_shape(i):
                n *= s
            cores.append(torch.empty(n, dtype=torch.float64, device="cuda"))
        return cores

    def assemble(self, cores=None, stream=None, check_status=True):
        cores = self.alloc_cores() if cores is None else cores
        ptrs = (C.c_void_p * self.num_nodes)(*[C.c_void_p(c.data_ptr()) for c in cores])
        st = lib.ttnn_assemble(self.handle, ptrs, stream_ptr(stream))
        if check_status:
            check(st)
        return cores if check_status else (cores, st)

    def assemble_async(self, cores=None, stream=None):
        """Enqueue the recovery phase without waiting; the numerical status is kept
        (sticky) until assemble_status()."""
        cores = self.alloc_cores() if cores is None else cores
        ptrs = (C.c_void_p * self.num_nodes)(*[C.c_void_p(c.data_ptr()) for c in cores])
        check(lib.ttnn_assemble_async(self.handle, ptrs, stream_ptr(stream)))
        return cores

    def assemble_status(self, stream=None, check_status=True):
        """Status of every assembly since the last query (waits for the stream)."""
        st = lib.ttnn_assemble_status(self.handle, stream_ptr(stream))
        if check_status:
            check(st)
        return st

    def assemble_status_async(self, h_status, stream=None):
        """Enqueue the status query into `h_status`, a pinned int32 CPU tensor of one
        element (0 = sound); read it after the stream has passed this call."""
        if not (isinstance(h_status, torch.Tensor) and h_status.dtype == torch.int32 and h_status.numel() >= 1
                and h_status.is_pinned()):
            raise TypeError("h_status must be a pinned int32 CPU tensor with at least one element")
        check(lib.ttnn_assemble_status_async(self.handle, C.c_void_p(h_status.data_ptr()), stream_ptr(stream)))

    def reconstruct(self, cores, out=None, out_dtype=F64, stream=None):
        n = 1
        for s in self.dims:
            n *= s
        if out is None:
            out = torch.empty(n, dtype=TORCH_DTYPE[out_dtype], device="cuda")
        ptrs = (C.c_void_p * self.num_nodes)(*[C.c_void_p(c.data_ptr()) for c in cores])
        check(lib.ttnn_reconstruct(self.handle, ptrs, C.c_void_p(out.data_ptr()), out_dtype, stream_ptr(stream)))
        return out


def diff_norms(a, b, stream=None):
    """(||a - b||^2, ||b||^2) computed on the GPU; a any plan dtype, b float64."""
    out = (C.c_double * 2)()
    if a.dtype not in (torch.float64, torch.float32, torch.bfloat16):
        raise TypeError(f"a has dtype {a.dtype}; expected float64, float32 or bfloat16")
    dt = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}[a.dtype]
    check_block(b, torch.float64, (a.numel(),), 1)
    check_block(a, a.dtype, (b.numel(),), 1)
    check(lib.ttnn_diff_norms(C.c_void_p(a.data_ptr()), dt, C.c_void_p(b.data_ptr()), a.numel(), out,
                              stream_ptr(stream)))
    return out[0], out[1]


def update_batched(items, stream=None):
    """items: list of (plan, block, extent, offset, alpha); see ttnn_sketch_update_batched."""
    arr = (UpdateDesc * max(1, len(items)))()
    keep = []
    for i, (plan, block, extent, offset, alpha) in enumerate(items):
        strides = view_strides(block, extent, plan.d)
        check_block(block, plan.torch_dtype, extent, plan.d, strides)
        if len(offset) != plan.d:
            raise ValueError(f"item {i}: offset has {len(offset)} modes, the tensor has {plan.d}")
        arr[i].plan = plan.handle
        arr[i].d_block = C.c_void_p(block.data_ptr())
        for mu in range(plan.d):
            arr[i].offset[mu] = int(offset[mu])
            arr[i].extent[mu] = int(extent[mu])
            arr[i].strides[mu] = 0 if strides is None else int(strides[mu])
        arr[i].alpha = float(alpha)
        keep.append(block)
    check(lib.ttnn_sketch_update_batched(len(items), arr, stream_ptr(stream)))
