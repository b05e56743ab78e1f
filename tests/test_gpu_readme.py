"""The Python example of README.md, run as written on the GPU, with checks
of what it computes: the documented use of the binding stays working."""

import os
import re

import numpy as np
import pytest
import torch

from gpu_common import require_gpu

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_example_runs():
    require_gpu()
    with open(os.path.join(ROOT, "README.md")) as fh:
        blocks = re.findall(r"```python\n(.*?)```", fh.read(), re.S)
    assert len(blocks) == 1
    env = {}
    exec(compile(blocks[0], "README.md", "exec"), env)
    torch.cuda.synchronize()
    w, tree, src, dirs = env["w"], env["tree"], env["src"], env["dirs"]
    S, Dn = src.shape[0], dirs.shape[0]
    assert env["N"].shape == (S, Dn) and env["A"].shape == (S, Dn)
    assert torch.isfinite(env["N"]).all()
    # the autograd path and the fused pass give the same N, and gradients of
    # the same size and sign (both losses are sums of positive weights times A)
    grad = env["rho"].grad
    assert grad is not None and grad.shape == (w.tree.n,)
    g = env["g"]
    assert g.shape == (w.tree.n,) and bool((g <= 0).all()) and bool((grad <= 0).all())
    out = env["out"]
    assert out["av_eff"].shape == (S,) and out["beta"].shape == (S, 3)
    assert bool(torch.isfinite(out["av_eff"]).all())
    keys, levels, values = env["keys"], env["levels"], env["values"]
    assert keys.numel() == levels.numel() == values.numel() == env["tree2"].n
    # the constructed leaves tile the 64^3 grid
    assert int((8 ** (6 - levels.to(torch.int64))).sum()) == 64 ** 3
    assert np.isclose(float((values * 8.0 ** (6 - levels.to(torch.float64))).sum()),
                      float(env["grid"].sum()), rtol=1e-10)
