"""mf_integrand_noalloc: the integrand at explicit points with its point lists
in the library's fixed device array, against mf_integrand (same kernels, so
bit-identical results), on two calls in a row, the second with fewer points;
size and process limits."""
import numpy as np
import pytest

import seeded_inputs as si
from gpu_util import to_dev_soa

pytestmark = pytest.mark.gpu


def _proc(name, **kw):
    import paper_2105_10529_amd as mf

    return mf.Process(mf.Config(process=name, **kw))


@pytest.mark.parametrize("name,prec,ng,sizes", [
    ("gg>ttxg", "fp64", 1, (1_200_000, 70_001)),   # several chunks per block, then one ragged chunk
    ("gg>ttxgg", "fp32", 2, (300_001, 4_097)),
    ("gg>ttxgg", "fp64", 2, (20_000, 513)),
    ("gg>ttx", "fp64", 0, (9_999, 1)),
])
def test_noalloc_matches_integrand(name, prec, ng, sizes):
    import torch

    # g g -> t t~ g g with the in-register colour form (single integrand kernel)
    kw = {"dr_min": 0.4, "colour_form": 1} if ng == 2 else {}
    p = _proc(name, precision=prec, **kw)
    for k, n in enumerate(sizes):
        print(f"noalloc {name} {prec} n={n}", flush=True)
        x = si.points_above_threshold(n, si.ndim(ng), 13000.0, 173.0, seed=900 + k)
        u = to_dev_soa(x)
        ref = p.integrand(u)
        w = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        p.integrand_noalloc(u, w)
        torch.cuda.synchronize()
        a, b = w.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(a, b), (n, int(np.sum(a != b)))
        assert np.count_nonzero(a) > 0


def test_noalloc_limits():
    import torch

    import paper_2105_10529_amd as mf

    p = _proc("gg>ttxg")
    n = mf.NOALLOC_MAX_POINTS + 1
    u = torch.full((7, n), 0.5, dtype=torch.float64, device="cuda")
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    with pytest.raises(mf.MFError, match="at most"):
        p.integrand_noalloc(u, w)
    for name, d, kw in (("gg>ttxggg", 13, {}), ("gg>ttxgg", 10, {"colour_form": 2})):
        p2 = _proc(name, precision="fp32", dr_min=0.4, **kw)
        u2 = torch.full((d, 8), 0.5, dtype=torch.float64, device="cuda")
        w2 = torch.empty(8, dtype=torch.float64, device="cuda")
        with pytest.raises(mf.MFError, match="workspace"):
            p2.integrand_noalloc(u2, w2)
