"""Khatri-Rao structured sketches of TTN-format tensors on the GPU (Sec. 7), through the
C ABI, against the oracle:

* the per-mode factors bit for bit (same counter-based generator, own tags);
* every accumulated sketch (Omega_t, Psi_t, leaf R_t, root Psi) element by element
  against the dense definition (oracle.sketch of the dense tensor with the dense
  Khatri-Rao maps) on the trees of Fig. 1, ((1,2),(3,4)), (((1,2),3),(4,5)) and one with
  a multi-mode leaf, at the FP64 tolerance;
* streaming: two scaled updates against the oracle sum; a caller's scratch against the
  pool's, bit for bit; dense updates refused;
* exact recovery of a TTN of rank <= r (GPU recovery and reconstruction);
* TTN inner products against the oracle's;
* the rounding workload of the paper's second experiment (order 6, tree of Fig. 1, mode
  size 500, TTN ranks 70 with quadratically decaying superdiagonal cores, p = 10): all
  sketches against the oracle's tree contraction, and the rounding error, computed by
  TTN inner products on the GPU, against the oracle's on its own recovery.
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import structured as S
from gpu_util import TOL, errs2, failures, sketch_errors
from workloads import synth as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2412_06111_amd as P
    return P


def dev_cores(cores):
    """Oracle-layout cores (keyed by node modes, column-major numpy) -> CUDA float64."""
    return {m: torch.from_numpy(np.ascontiguousarray(c.reshape(-1, order="F"))).cuda() for m, c in cores.items()}


def oracle_cores_by_modes(tree, oc):
    return {tree[v].modes: oc[v].reshape(O.core_shape(tree, v), order="F") for v in oc}


def host_cores(plan, cores):
    """GPU cores (list by caller id) -> dict keyed by node modes, numpy column-major shapes."""
    out = {}
    for i, c in enumerate(cores):
        out[plan.node_modes[i]] = c.cpu().numpy().reshape(plan.core_shape(i), order="F")
    return out


def test_factors_bit_exact(P):
    dims, r, p = (7, 5, 9, 4), 6, 3
    plan = P.Plan(O.T4, dims, r, p, variant="kr", seed=13)
    X, Y = S.factors(13, dims, r, p)
    for mu in range(4):
        assert np.array_equal(plan.read_factor(mu, 0).cpu().numpy(), X[mu])
        assert np.array_equal(plan.read_factor(mu, 1).cpu().numpy(), Y[mu])
    plan.close()


CASES = [
    ("toy", O.TOY, (9, 12, 7, 10, 8, 11), 5),
    ("t4", O.T4, (40, 33, 27, 50), 7),
    ("t5", O.T5, (13, 9, 16, 11, 10), 6),
    ("multileaf", ((frozenset({1, 2}), 3), (4, 5)), (6, 5, 9, 7, 8), 4),
]


@pytest.mark.parametrize("name,spec,dims,s", CASES, ids=[c[0] for c in CASES])
def test_structured_sketch_matches_dense_definition(P, name, spec, dims, s):
    r, p = 6, 3
    print(f"structured sketch {name} dims={dims} s={s}", flush=True)
    cores = W.gaussian_ttn_cores(spec, dims, s, seed=21)
    T = W.ttn_dense(spec, dims, cores)
    tree = O.Tree(spec, dims, r, p)
    X, Y = S.factors(5, dims, r, p)
    want = O.sketch(T, tree, S.kr_drms(tree, X, Y), "ttnn")
    plan = P.Plan(spec, dims, r, p, variant="kr", seed=5)
    plan.update_ttn(dev_cores(cores), s)
    torch.cuda.synchronize()
    bad = failures(sketch_errors(plan, tree, want), TOL["f64"])
    assert not bad, bad
    plan.close()


def test_streaming_alpha_and_scratch(P):
    spec, dims, r, p = O.TOY, (8, 6, 9, 7, 5, 6), 5, 2
    A = W.gaussian_ttn_cores(spec, dims, 4, seed=1)
    B = W.gaussian_ttn_cores(spec, dims, 3, seed=2)
    tree = O.Tree(spec, dims, r, p)
    X, Y = S.factors(3, dims, r, p)
    sa, sb = S.ttn_sketch(A, tree, X, Y), S.ttn_sketch(B, tree, X, Y)
    want = {k: {t: 0.5 * sa[k][t] - 2.0 * sb[k][t] for t in sa[k]} for k in ("R", "Omega", "Psi")}
    pool = P.Plan(spec, dims, r, p, variant="kr", seed=3)
    mine = P.Plan(spec, dims, r, p, variant="kr", seed=3)
    dA, dB = dev_cores(A), dev_cores(B)
    pool.update_ttn(dA, 4, alpha=0.5)
    pool.update_ttn(dB, 3, alpha=-2.0)
    need = max(mine.update_ttn_work_bytes(4), mine.update_ttn_work_bytes(3))
    work = torch.empty(need, dtype=torch.uint8, device="cuda")
    mine.update_ttn(dA, 4, alpha=0.5, work=work)
    mine.update_ttn(dB, 3, alpha=-2.0, work=work)
    torch.cuda.synchronize()
    bad = failures(sketch_errors(pool, tree, want), TOL["f64"])
    assert not bad, bad
    from paper_2412_06111_amd import SK_OMEGA, SK_PSI
    for i in range(pool.num_nodes):
        kinds = (SK_PSI,) if i == 0 else (SK_OMEGA, SK_PSI)
        for k in kinds:
            assert torch.equal(pool.read_sketch(i, k).view(torch.int64), mine.read_sketch(i, k).view(torch.int64))
    with pytest.raises(P.TTNNError):                     # too small a scratch is refused
        mine.update_ttn(dA, 4, work=work[:256])
    with pytest.raises(P.TTNNError):                     # dense updates are refused
        mine.update(torch.zeros(int(np.prod(dims)), dtype=torch.float64, device="cuda"))
    pool.close()
    mine.close()


@pytest.mark.parametrize("spec,dims", [(O.TOY, (10, 8, 12, 9, 7, 11)), (O.T5, (14, 10, 12, 9, 13))])
def test_exact_recovery_of_low_rank_ttn(P, spec, dims):
    s, r, p = 3, 4, 2
    cores = W.gaussian_ttn_cores(spec, dims, s, seed=8)
    T = W.ttn_dense(spec, dims, cores)
    plan = P.Plan(spec, dims, r, p, variant="kr", seed=9)
    plan.update_ttn(dev_cores(cores), s)
    gc = plan.assemble()
    That = plan.reconstruct(gc).cpu().numpy()
    ref = W.flat_colmajor(T)
    assert np.linalg.norm(That - ref) <= 1e-10 * np.linalg.norm(ref)
    plan.close()


def test_ttn_dot_matches_oracle(P):
    spec, dims = O.TOY, (9, 7, 8, 10, 6, 7)
    A = W.gaussian_ttn_cores(spec, dims, 4, seed=3)
    B = W.gaussian_ttn_cores(spec, dims, {m: 2 + len(m) % 3 for m in [n[1] for n in W.tree_spec_nodes(spec)]}, seed=4)
    tree = O.Tree(spec, dims, 4, 0)
    rb = {n[1]: 2 + len(n[1]) % 3 for n in W.tree_spec_nodes(spec)}
    plan = P.Plan(spec, dims, 4, 2, variant="kr", seed=1)
    got = plan.ttn_dot(dev_cores(A), 4, dev_cores(B), rb)
    want = S.ttn_dot(tree, A, B)
    dense = float(np.sum(W.ttn_dense(spec, dims, A) * W.ttn_dense(spec, dims, B)))
    scale = np.sqrt(S.ttn_dot(tree, A, A) * S.ttn_dot(tree, B, B))
    assert abs(got - want) <= 1e-12 * scale and abs(want - dense) <= 1e-12 * scale
    plan.close()


def rounding_input(n=500, s=70, seed=0):
    sigma = 1.0 / np.arange(1, s + 1) ** 2
    return W.decaying_ttn_cores(O.TOY, (n,) * 6, s, sigma, seed=seed)


@pytest.fixture(scope="module")
def rounding():
    return rounding_input()


@pytest.mark.parametrize("r", [16, 48])
def test_rounding_workload_parity(P, rounding, r):
    p, n, s = 10, 500, 70
    dims = (n,) * 6
    print(f"rounding workload parity r={r}", flush=True)
    tree = O.Tree(O.TOY, dims, r, p)
    X, Y = S.factors(2, dims, r, p)
    want = S.ttn_sketch(rounding, tree, X, Y)
    plan = P.Plan(O.TOY, dims, r, p, variant="kr", seed=2)
    dc = dev_cores(rounding)
    plan.update_ttn(dc, s)
    torch.cuda.synchronize()
    bad = failures(sketch_errors(plan, tree, want), TOL["f64"])
    assert not bad, bad
    # rounding error ||T - T_r|| / ||T|| by TTN inner products, GPU against oracle
    gc = plan.assemble()
    rr = plan.core_ranks()
    tt = plan.ttn_dot(dc, s, dc, s)
    tr = plan.ttn_dot(dc, s, gc, rr)
    rrd = plan.ttn_dot(gc, rr, gc, rr)
    e_gpu = np.sqrt(max(tt - 2 * tr + rrd, 0.0) / tt)
    oc, _ = O.assemble(want, tree)
    ocm = oracle_cores_by_modes(tree, oc)
    ott = S.ttn_dot(tree, rounding, rounding)
    e_or = np.sqrt(max(ott - 2 * S.ttn_dot(tree, rounding, ocm) + S.ttn_dot(tree, ocm, ocm), 0.0) / ott)
    print(f"r={r}: rounding error gpu {e_gpu:.6e} oracle {e_or:.6e}", flush=True)
    assert abs(e_gpu - e_or) <= 1e-3 * e_or, (e_gpu, e_or)
    # the GPU cores themselves against the oracle's (same recovery, FP64)
    hc = host_cores(plan, gc)
    for m in ocm:
        e = errs2(hc[m], ocm[m])
        assert e[0] <= 1e-8, (m, e)
    plan.close()
