"""The Python example in README.md runs as written (factorize on the device,
plan, batch render) and sampled rows match the oracle's per-sample
definition within the FP32 render bound."""
import os
import re

import numpy as np
import pytest

import fp32bound
import oracle

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_example(dev):
    import torch
    text = open(os.path.join(ROOT, "README.md")).read()
    code = re.search(r"```python\n(.*?)```", text, re.S).group(1)
    ns = {}
    exec(compile(code, "README.md", "exec"), ns)
    torch.cuda.synchronize()
    out, out_off, jobs, srcs, fac, plan, lens = (ns[k] for k in ("out", "out_off", "jobs", "srcs", "fac", "plan",
                                                                 "lens"))
    r = fac["f"].astype(np.float32)
    k = fac["p"].shape[1]
    for j in (0, 5, len(jobs) - 1):
        s, f = jobs[j]
        n = plan.out_len(lens[s])
        t = np.array([0, 1, 1000, 500000, n - 1], dtype=np.int64)
        got = out[torch.from_numpy(out_off[j] + t).to(dev)].cpu().numpy().astype(np.float64)
        g = fac["g"][f].astype(np.float32)
        ref = oracle.sparse_render_points(r, srcs[s], fac["p"][f], g, t)
        bound = fp32bound.render_bound(r, srcs[s], fac["p"][f], g, t, k)
        assert np.all(np.abs(got - ref) <= bound), (j, got, ref)
    ns["batch"].close()
    plan.close()
