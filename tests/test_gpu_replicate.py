"""The replication harness at small n: the paper's bricks, random initial
guess and C-norm stopping reproduce the observations of Sections 2-4 on the
GPU, and the harness's solves agree with the oracle's."""
import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def test_linear_series_shapes():
    from paper_1212_6680_amd import replicate as R
    p = R.linear_point(torch, 32)
    assert p["shape"] == [32, 512, 32]
    # Figs. 1-2: equations (1) and (2) give the same CG without a preconditioner
    a, b = p["cg1_noprec"], p["cg2_noprec"]
    assert a["iters"] == b["iters"]
    assert b["rel_res_c"] == pytest.approx(a["rel_res_c"], rel=1e-3)
    assert p["sd_noprec"]["rel_res_c"] > 10 * a["rel_res_c"]          # SD is far behind
    # Figs. 3-4: with balanced SMG the two PCG variants coincide, PSD needs a few more
    assert abs(p["pcg_11"]["iters"] - p["fpcg_11"]["iters"]) <= 1
    assert p["fpcg_11"]["iters"] <= p["psd_11"]["iters"] <= p["fpcg_11"]["iters"] + 4
    # Figs. 5-7: without post-smoothing standard PCG stalls; flexible PCG and PSD converge, close together
    assert p["pcg_10"]["status"] == 1 and p["pcg_10"]["rel_res_c"] > R.RTOL_C      # 100 iterations not enough
    assert p["fpcg_10"]["status"] == 0 and p["psd_10"]["status"] == 0
    assert p["fpcg_10"]["iters"] <= p["psd_10"]["iters"] <= p["fpcg_10"]["iters"] + 2
    assert p["fpcg_10"]["rel_res_c"] <= R.RTOL_C
    # a (1,0) iteration is cheaper than a (1,1) iteration
    per = lambda r: r["s"] / r["iters"]
    assert per(p["fpcg_10"]) < per(p["fpcg_11"])


def test_orientation_of_the_brick_matters_little():
    from paper_1212_6680_amd import replicate as R
    a = R.linear_point(torch, 16, paper_orientation=True)
    b = R.linear_point(torch, 16)
    assert a["shape"] == [256, 16, 16]
    for k in ("fpcg_10", "psd_10", "pcg_11", "fpcg_11"):
        assert abs(a[k]["iters"] - b[k]["iters"]) <= 2, k


def test_lobpcg_m1_series():
    from paper_1212_6680_amd import replicate as R
    p = R.lobpcg_point(torch, 8)
    assert p["shape"] == [16, 32, 16]
    for k in ("lobpcg_11", "lobpcg_10"):
        assert p[k]["status"] == 0 and p[k]["rel_eig_err"] <= 1e-8
    # Section 4: without post-smoothing a few more, cheaper iterations
    assert p["lobpcg_10"]["iters"] >= p["lobpcg_11"]["iters"]


@pytest.mark.parametrize("meth,pp", [("fpcg", (1, 0)), ("psd", (1, 0)), ("pcg", (1, 1))])
def test_brick_solve_matches_oracle(meth, pp):
    """A mapped brick (8, 128, 8), random x0, C-norm stopping at the harness's
    threshold: iteration counts within one of the oracle's, solutions to 1e-6."""
    from paper_1212_6680_amd import replicate as R
    from paper_1212_6680_amd.smg import SMG
    shape = R.brick("linear", 8)
    N = int(np.prod(shape))
    c = (1.0, 1.0, 1.0)
    b = synth.rhs(*shape, 1)
    x0 = synth.uniform_pm1(2, N)
    ref = O.krylov({"fpcg": O.FPCG, "psd": O.PSD, "pcg": O.PCG}[meth], b, shape, c, O.SMG(shape, c, *pp), x0=x0,
                   rtol=R.RTOL_C, stop="c")
    x, info = getattr(SMG(shape, c, *pp), meth)(torch.from_numpy(b).cuda(), torch.from_numpy(x0.copy()).cuda(),
                                               rtol=R.RTOL_C, stop="c")
    assert ref.status == 0 and info.status == 0
    assert abs(info.iters - ref.iters) <= 1
    assert np.linalg.norm(x.cpu().numpy() - ref.x) <= 1e-6 * np.linalg.norm(ref.x)


def test_theory_point_small():
    from paper_1212_6680_amd import replicate as R
    p = R.theory_point(torch, 6, iters=40)
    a, b = p["smg11"], p["smg10"]
    assert 0 < a["delta_min"] < b["delta_min"] < 1.0
    assert a["theorem2_delta"] == pytest.approx(a["delta_at_prescaling"], rel=0.05)
    for r in (a, b):
        assert r["psd_max_step_ratio"] <= r["delta_min"] * 1.05
