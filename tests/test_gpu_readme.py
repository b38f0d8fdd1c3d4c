"""The usage example of README.md runs as written (whole-tensor update in the searched
visiting order, recovery, error; then the same tensor streamed as two boxes read in
place plus a rank-1 term), and the streamed sketches equal those of the whole tensor
plus the term."""
import os
import re

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_example_runs():
    import paper_2412_06111_amd as P
    with open(os.path.join(ROOT, "README.md")) as f:
        code = re.search(r"```python\n(.*?)```", f.read(), re.S).group(1)
    print("readme example", flush=True)
    ns = {}
    exec(compile(code, "README.md", "exec"), ns)
    err2, norm2, plan = ns["err2"], ns["norm2"], ns["plan"]
    assert np.isfinite(err2) and norm2 > 0
    # the streamed sketches against the whole tensor plus the term, sketched again
    T, a, spec, dims = ns["T"], ns["a"], ns["spec"], ns["dims"]
    streamed = [plan.read_sketch(i, P.SK_PSI).cpu().numpy() for i in range(plan.num_nodes)]
    ref = P.Plan(spec, dims, 32, 16, variant="sttnn", dtype="f32", seed=7, visit=ns["visit"])
    ref.update(T)
    ref.update_rank1(a, alpha=0.5)
    for i in range(plan.num_nodes):
        want = ref.read_sketch(i, P.SK_PSI).cpu().numpy()
        assert np.linalg.norm(streamed[i] - want) <= 1e-5 * np.linalg.norm(want), plan.node_modes[i]
    ref.close()
    plan.close()
    del ns
    torch.cuda.empty_cache()
