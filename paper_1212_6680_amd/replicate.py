"""Replication of the paper's experiments on one MI355X (Sections 2-5, Figs. 1-9).

Workloads, as the paper's `struct` runs set them up (Section 2): the 7-point
negative Laplacian with unit grid size and homogeneous Dirichlet boundary on
bricks that grow with n -- 16n x n x n for the linear solves (the shared-memory
panels: 16 processors with an n^3 box each, stacked along the first axis) and
4n x 2n x 2n for LOBPCG with m = 1 (Section 4) -- a pseudo-random initial
guess, and the iteration stopped on the ratio ||r||_C / ||b||_C that the
figures plot, C being the preconditioner.

Readings where the paper is silent (stated again in the design notes):
* Orientation.  The library's line solves run along x and cap lines at 512
  points, while 16n reaches 2880.  The operator is isotropic, so the brick is
  the same matrix with its long axis along y instead: grid (n, 16n, n) (and
  (2n, 4n, 2n) for LOBPCG).  z, the semicoarsened axis, stays short as in the
  paper's layout; where 16n <= 512 the paper's own orientation (16n, n, n) is
  run too and both are reported.
* Right-hand side and initial guess: b and x0 i.i.d. uniform on [-1, 1) from
  seeded counter-based streams (the paper says only "pseudo-random").
* Stopping: the plotted quantity falls to ~1e-16 (Fig. 5); read as the squared
  ratio (T r, r) / (T b, b), the stopping points of Fig. 5 put its threshold
  in [4.7e-16, 2.1e-15); the runs stop when sqrt|(T r, r)| / sqrt|(T b, b)|
  <= 3.16e-8, i.e. at a squared ratio of 1e-15.  Without a preconditioner
  (Figs. 1-2) C = I and the cap is 100 iterations, as in the paper.
* LOBPCG stops when ||A x - lambda x|| / (lambda ||x||) <= 1e-8 (the paper's
  BLOPEX tolerance is not given).

Usage:
    python -m paper_1212_6680_amd.replicate --n 10,20,...,180 --json out.json --md out.md
Every number comes from the library's kernels through the binding; the
harness only sets up inputs, times calls and tabulates.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

RTOL_C = 10 ** -7.5          # squared C-norm ratio 1e-15
RTOL_EIG = 1e-8
CG_CAP = 100


def brick(kind: str, n: int, paper_orientation: bool = False):
    """(nx, ny, nz) of the paper's brick for this n."""
    if kind == "linear":
        return (16 * n, n, n) if paper_orientation else (n, 16 * n, n)
    if kind == "lobpcg":
        return (4 * n, 2 * n, 2 * n) if paper_orientation else (2 * n, 4 * n, 2 * n)
    raise ValueError(kind)


def _timed(torch, fn, reps=1):
    """(result of the last call, median seconds) after one warm-up call."""
    fn()
    ts, out = [], None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return out, float(np.median(ts))


def smallest_eig(shape, c=(1.0, 1.0, 1.0)):
    """Smallest eigenvalue of the Dirichlet 7-point operator on the brick."""
    return float(sum(4.0 * cc * np.sin(np.pi / (2.0 * (m + 1))) ** 2 for m, cc in zip(shape, c)))


def linear_point(torch, n, paper_orientation=False, reps=1, seed_b=1, seed_x=2, history=False):
    """Every linear-solve series of Figs. 1-7 at one n."""
    import synth
    from paper_1212_6680_amd.smg import SMG
    shape = brick("linear", n, paper_orientation)
    N = int(np.prod(shape))
    c = (1.0, 1.0, 1.0)
    b = torch.from_numpy(synth.rhs(*shape, seed_b)).cuda()
    x0 = torch.from_numpy(synth.uniform_pm1(seed_x, N)).cuda()
    x = torch.empty_like(b)
    out = {"n": n, "shape": list(shape), "dof": N}
    G11 = SMG(shape, c, 1, 1)

    def solve(G, meth, precond="smg", cap=500, rtol=RTOL_C, hist=False):
        def f():
            x.copy_(x0)
            return getattr(G, meth)(b, x, rtol=rtol, max_iter=cap, precond=precond, stop="c", history=hist)[1]
        info, sec = _timed(torch, f, reps)
        rec = {"iters": info.iters, "s": sec, "status": info.status, "rel_res_c": info.rel_res_c,
               "rel_res_c_squared": info.rel_res_c ** 2, "true_rel_res": info.true_rel_res}
        if hist:
            hc = np.array(info.history_c)
            rec["history_c_squared"] = (hc ** 2).tolist()
        return rec

    # Figs. 1-2: no preconditioner (C = I), capped at 100 iterations
    for name, meth in (("cg1", "pcg"), ("cg2", "fpcg"), ("sd", "psd")):
        out[f"{name}_noprec"] = solve(G11, meth, precond="none", cap=CG_CAP)
    # Figs. 3-4: balanced SMG (1,1)
    for meth in ("pcg", "fpcg", "psd"):
        out[f"{meth}_11"] = solve(G11, meth, hist=history)
    del G11
    # Figs. 5-7: SMG without post-smoothing (1,0); standard PCG capped at 100
    G10 = SMG(shape, c, 1, 0)
    for meth in ("pcg", "fpcg", "psd"):
        out[f"{meth}_10"] = solve(G10, meth, cap=CG_CAP if meth == "pcg" else 500, hist=history)
    del G10
    torch.cuda.empty_cache()
    return out


def lobpcg_point(torch, n, reps=1, seed=3):
    """Figs. 8-9: LOBPCG for the smallest eigenpair (m = 1) with SMG (1,1) and (1,0)."""
    import synth
    from paper_1212_6680_amd.smg import SMG
    shape = brick("lobpcg", n)
    N = int(np.prod(shape))
    X0 = torch.from_numpy(synth.block(N, 1, seed)).cuda()
    lam_exact = smallest_eig(shape)
    out = {"n": n, "shape": list(shape), "dof": N}
    for pp in ((1, 1), (1, 0)):
        G = SMG(shape, (1.0, 1.0, 1.0), *pp, max_nrhs=1)
        (lam, _, info), sec = _timed(torch, lambda: G.lobpcg(X0, rtol=RTOL_EIG, max_iter=200), reps)
        out[f"lobpcg_{pp[0]}{pp[1]}"] = {"iters": info.iters, "s": sec, "status": info.status,
                                         "rel_eig_err": abs(lam[0] - lam_exact) / lam_exact}
        del G
    torch.cuda.empty_cache()
    return out


def theory_point(torch, n, iters=60, seed=4):
    """Section 5 at one n of the linear bricks: min_c ||I - c A T||_{A^{-1}} for
    (1,1) and (1,0), Theorem 2's prescaled delta for (1,1), and the worst PSD
    contraction of ||r||_{A^{-1}} per step against an exact solution from a
    tight flexible-PCG solve."""
    import synth
    from paper_1212_6680_amd.smg import SMG
    shape = brick("linear", n)
    N = int(np.prod(shape))
    c = (1.0, 1.0, 1.0)
    v0 = torch.from_numpy(synth.uniform_pm1(seed, N)).cuda()
    b = torch.from_numpy(synth.rhs(*shape, 1)).cuda()
    out = {"n": n, "shape": list(shape)}
    G11, G10, G01 = SMG(shape, c, 1, 1), SMG(shape, c, 1, 0), SMG(shape, c, 0, 1)
    xs, _ = G11.fpcg(b, rtol=1e-13)
    lo, hi = G11.spectrum(v0, iters=iters)
    kappa = hi / lo
    out["smg11"] = {"lambda_min": lo, "lambda_max": hi, "theorem2_delta": (kappa - 1) / (kappa + 1),
                    "delta_at_prescaling": G11.delta(2.0 / (lo + hi), v0, iters=iters)}
    for name, G, Gt in (("smg11", G11, G11), ("smg10", G10, G01)):
        cb, d = G.delta_min(v0, 0.5, 2.0, 1e-3, iters=iters, transpose=Gt)
        _, info = G.psd(b, rtol=1e-11, xstar=xs)
        e = np.array(info.err_a)
        ok = e[:-1] > 1e-8
        ratio = e[1:][ok] / e[:-1][ok]
        out.setdefault(name, {}).update({"c_best": cb, "delta_min": d, "psd_max_step_ratio": float(ratio.max()),
                                         "psd_mean_step_ratio": float(np.exp(np.log(ratio).mean()))})
    del G11, G10, G01
    torch.cuda.empty_cache()
    return out


def markdown(res) -> str:
    """The figures' series as tables."""
    lines = []
    lin = res.get("linear", [])
    if lin:
        lines += ["### Figs. 1-2: unpreconditioned CG (100-iteration cap)", "",
                  "| n | DoF | CG(1) ms/it | CG(2) ms/it | overhead | CG(1) final | CG(2) final | SD final |",
                  "|---|---|---|---|---|---|---|---|"]
        for p in lin:
            a, b, sd = p["cg1_noprec"], p["cg2_noprec"], p["sd_noprec"]
            pa, pb = 1e3 * a["s"] / max(a["iters"], 1), 1e3 * b["s"] / max(b["iters"], 1)
            lines.append(f"| {p['n']} | {p['dof']} | {pa:.3f} | {pb:.3f} | {100 * (pb / pa - 1):+.0f}% | "
                         f"{a['rel_res_c']:.2e} | {b['rel_res_c']:.2e} | {sd['rel_res_c']:.2e} |")
        lines += ["", "### Figs. 3-4 and 6-7: SMG-preconditioned solves (iterations / ms)", "",
                  "| n | PCG(1,1) | FPCG(1,1) | PSD(1,1) | PCG(1,0) | FPCG(1,0) | PSD(1,0) | FPCG saving (1,0) vs (1,1) |",
                  "|---|---|---|---|---|---|---|---|"]
        for p in lin:
            cells = []
            for k in ("pcg_11", "fpcg_11", "psd_11", "pcg_10", "fpcg_10", "psd_10"):
                r = p[k]
                tag = "" if r["status"] == 0 else " (no conv.)"
                cells.append(f"{r['iters']}{tag} / {1e3 * r['s']:.1f}")
            save = 1 - p["fpcg_10"]["s"] / p["fpcg_11"]["s"]
            lines.append(f"| {p['n']} | " + " | ".join(cells) + f" | {100 * save:.0f}% |")
    f5 = res.get("fig5")
    if f5:
        lines += ["", f"### Fig. 5: squared C-norm ratio per iteration, n = {f5['n']} (grid {f5['shape']})", "",
                  "| k | PCG(1,0) | PSD(1,0) | FPCG(1,0) |", "|---|---|---|---|"]
        hs = [f5[k]["history_c_squared"] for k in ("pcg_10", "psd_10", "fpcg_10")]
        for k in range(max(len(h) for h in hs)):
            lines.append(f"| {k} | " + " | ".join(f"{h[k]:.3e}" if k < len(h) else "" for h in hs) + " |")
    lob = res.get("lobpcg", [])
    if lob:
        lines += ["", "### Figs. 8-9: LOBPCG m = 1 on 4n x 2n x 2n (iterations / ms)", "",
                  "| n | DoF | (1,1) | (1,0) | saving | eig. error (1,0) |", "|---|---|---|---|---|---|"]
        for p in lob:
            a, b = p["lobpcg_11"], p["lobpcg_10"]
            lines.append(f"| {p['n']} | {p['dof']} | {a['iters']} / {1e3 * a['s']:.1f} | {b['iters']} / "
                         f"{1e3 * b['s']:.1f} | {100 * (1 - b['s'] / a['s']):.0f}% | {b['rel_eig_err']:.1e} |")
    th = res.get("theory", [])
    if th:
        lines += ["", "### Section 5: assumption (4), bound (3), Theorem 2", "",
                  "| n | (1,1) delta_min | (1,1) Thm 2 delta | (1,1) PSD worst step | (1,0) delta_min | (1,0) c_best | (1,0) PSD worst step |",
                  "|---|---|---|---|---|---|---|"]
        for p in th:
            a, b = p["smg11"], p["smg10"]
            lines.append(f"| {p['n']} | {a['delta_min']:.4f} | {a['theorem2_delta']:.4f} | "
                         f"{a['psd_max_step_ratio']:.4f} | {b['delta_min']:.4f} | {b['c_best']:.3f} | "
                         f"{b['psd_max_step_ratio']:.4f} |")
    orient = res.get("orientation", [])
    if orient:
        lines += ["", "### Orientation check: (16n, n, n) as in the paper vs (n, 16n, n)", "",
                  "| n | FPCG(1,0) it. paper / mapped | PSD(1,0) | PCG(1,1) |", "|---|---|---|---|"]
        for p in orient:
            a, b = p["paper"], p["mapped"]
            lines.append(f"| {p['n']} | {a['fpcg_10']['iters']} / {b['fpcg_10']['iters']} | "
                         f"{a['psd_10']['iters']} / {b['psd_10']['iters']} | "
                         f"{a['pcg_11']['iters']} / {b['pcg_11']['iters']} |")
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n", default="10,20,30,40,50,60,70,80,90,100,110,120,130,140,150,160,170,180")
    ap.add_argument("--lobpcg-n", default="10,20,30,40,50,60,70,80,90,100,110,120")
    ap.add_argument("--theory-n", default="8,16,24,32")
    ap.add_argument("--orientation-n", default="8,16,24,32")
    ap.add_argument("--fig5-n", type=int, default=80)
    ap.add_argument("--reps", type=int, default=1)
    ap.add_argument("--json", default=None)
    ap.add_argument("--md", default=None)
    a = ap.parse_args(argv)
    import torch
    ints = lambda s: [int(v) for v in s.split(",") if v]
    res = {"rtol_c": RTOL_C, "rtol_eig": RTOL_EIG, "linear": [], "lobpcg": [], "theory": [], "orientation": []}
    for n in ints(a.n):
        res["linear"].append(linear_point(torch, n, reps=a.reps))
        print(f"linear n={n} done", flush=True)
    if a.fig5_n:
        res["fig5"] = linear_point(torch, a.fig5_n, history=True)
        print("fig5 done", flush=True)
    for n in ints(a.orientation_n):
        if 16 * n <= 512:
            res["orientation"].append({"n": n, "paper": linear_point(torch, n, paper_orientation=True),
                                       "mapped": linear_point(torch, n)})
    for n in ints(a.lobpcg_n):
        res["lobpcg"].append(lobpcg_point(torch, n, reps=a.reps))
        print(f"lobpcg n={n} done", flush=True)
    for n in ints(a.theory_n):
        res["theory"].append(theory_point(torch, n))
        print(f"theory n={n} done", flush=True)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(res, f)
    md = markdown(res)
    if a.md:
        with open(a.md, "w") as f:
            f.write(md)
    print(md)
    return res


if __name__ == "__main__":
    main()
