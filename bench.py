"""Benchmark: flexible-PCG with the SMG(1,0) preconditioner to 1e-8 on a 256^3 brick.

One step = one fpcg_solve call: Algorithm 1 with beta from equation (2) and
one SMG V-cycle without post-smoothing per iteration (the paper's
"post-smoothing off" mode, Section 3), on the 7-point Dirichlet Laplacian of
the unit cube with 256 interior points per axis (c = 257^2), b ~ U[-1, 1)
from seed 2, x0 = 0, stopping at ||r||_2/||b||_2 <= 1e-8.  Inputs are resident
in HBM before the timed region; setup is timed separately.

Prints one JSON line.  value = seconds per solve (time to 1e-8).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "FPCG-SMG time to 1e-8 rel. residual at 256^3; SMG V-cycle GDoF/s; % HBM roofline"
KERNEL_SRCS = [os.path.join(ROOT, "paper_1212_6680_amd", "csrc", f) for f in ("smg_kernels.hip", "smg_fused.hip")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_256.txt")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


KERNEL_NAMES = {
    "down2": "k2_down_march / k2_down_reg / k2_down (fused pre-smoothing + residual + restriction of a 2D level)",
    "coarse2": "k2_coarse (LDS-resident 2D sub-cycle)",
    "chain2": "k2_chain (2D prolongation chain + 3D correction)",
    "up2": "k2_up (fused prolongation + post-smoothing)",
    "chain3": "k3_chain (3D prolongation chain)",
    "resid3": "k_resid3v (3D colour residual)",
    "restrict3": "k_restrict3_march / k_restrict3 (3D residual + restriction)",
    "prolong3": "k_prolong3", "line_relax": "k_line_relax", "restrict2": "k_restrict2",
    "prolong2": "k_prolong2", "correct3": "k_correct3",
}


def read_traffic(family, schedule=None):
    """HBM bytes per launch of `family` from the committed counter summary, or
    None when it is missing, covers another kernel, was taken on a different
    kernel source, or on another V-cycle schedule than `schedule`."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_source_hash() or kv.get("family") != family:
        return None
    if schedule is not None and (kv.get("schedule_l0") != str(schedule[0]) or
                                 kv.get("schedule_coarse_lds") != str(schedule[1]) or
                                 kv.get("schedule_march_waves") != str(schedule[2])):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def other_configs(torch, dev, learned=True):
    """The other workloads of the hot path, each timed once after a warm-up:
    LOBPCG at 128^3, FPCG at 384^3 with the SMG preconditioner in FP64, FP32
    and BF16 storage, the 48 uneven boxes, and the learned post-smoother."""
    import synth
    from paper_1212_6680_amd.smg import SMG

    res = lobpcg_configs(torch, dev)
    res.update(precision_configs(torch, dev))
    res["batch_48_uneven"] = batch_config(torch, dev)
    res["varcoef_256"] = varcoef_config(torch, dev)
    if learned:
        res["learned_256"] = learned_config(torch, dev)
    return res


def precision_configs(torch, dev):
    """FPCG at 384^3 with the SMG preconditioner in FP64, FP32 and BF16 storage."""
    import synth
    from paper_1212_6680_amd.smg import SMG

    res = {}
    n = 384
    shape, c = (n, n, n), ((n + 1.0) ** 2,) * 3
    b = torch.from_numpy(synth.rhs(n, n, n, 5)).to(dev)
    x64 = None
    for prec in ("f64", "f32", "bf16"):
        G = SMG(shape, c, 1, 0, precision=prec)
        tune = G.autotune(b, reps=2)
        x = torch.empty_like(b)
        G.fpcg(b, x, rtol=1e-8, max_iter=3, zero_x0=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = G.fpcg(b, x, rtol=1e-8, max_iter=500, zero_x0=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if prec == "f64":
            x64 = x.clone()
        err = float(torch.linalg.vector_norm(x - x64) / torch.linalg.vector_norm(x64))
        # the V-cycle alone, and per kernel family: launches, ms and algorithmic
        # bytes per V-cycle (values stored in the precision's storage type)
        s = torch.empty_like(b)
        G.apply(b, s)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(10):
            G.apply(b, s)
        ev1.record()
        torch.cuda.synchronize()
        vms = ev0.elapsed_time(ev1) / 10
        fams = {}
        for fam in ("down2", "coarse2", "chain2", "chain3", "resid3", "restrict3"):
            nl, ms, by = G.profile_kernel(fam, b, reps=3)
            if nl:
                gbs = by / (ms * 1e-3) / 1e9
                fams[fam] = {"launches": nl, "ms": round(ms, 4), "mb": round(by / 1e6, 1),
                             "gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 3)}
        vbytes = sum(f["mb"] for f in fams.values()) * 1e6
        res[f"fpcg_384_smg_{prec}"] = {"s": dt, "iters": info.iters, "status": info.status,
                                       "true_rel_res": info.true_rel_res, "rel_err_vs_f64_solution": err,
                                       "vcycle_ms": vms, "vcycle_gdof_per_s": n ** 3 / (vms * 1e-3) / 1e9,
                                       "vcycle_hbm_frac": vbytes / (vms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                       "schedule": {"l0": tune.l0, "march_waves": tune.march_waves},
                                       "kernels_per_vcycle": fams}
        del G
    del b, x, x64
    torch.cuda.empty_cache()
    return res


def lobpcg_configs(torch, dev):
    """LOBPCG for the m = 16 and m = 64 smallest eigenpairs of the 128^3
    Laplacian (SMG(1,0) on the whole active block in one batched V-cycle),
    checked against the closed-form spectrum, with the Gram product's rate on
    the FP64 matrix cores."""
    import synth
    from paper_1212_6680_amd.smg import SMG

    def smallest_eigs(nn, cc, m):
        # Dirichlet Laplacian spectrum: sums of 4 c sin^2(k pi / (2 (n+1))) over the three axes
        k = np.arange(1, min(nn, m) + 1)
        l1 = 4.0 * cc * np.sin(k * np.pi / (2 * (nn + 1))) ** 2
        return np.sort((l1[:, None, None] + l1[None, :, None] + l1[None, None, :]).ravel())[:m]

    res = {}
    n = 128
    shape, c = (n, n, n), ((n + 1.0) ** 2,) * 3
    # balanced smoothing for comparison (Section 4: fewer iterations, dearer ones)
    G = SMG(shape, c, 1, 1, max_nrhs=16)
    X0 = torch.from_numpy(synth.block(n ** 3, 16, 3)).to(dev)
    G.lobpcg(X0, rtol=1e-8, max_iter=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lam, X, info = G.lobpcg(X0, rtol=1e-8, max_iter=400)
    torch.cuda.synchronize()
    res["lobpcg_128_m16_smg11"] = {"s": time.perf_counter() - t0, "iters": info.iters, "nconv": info.nconv,
                                   "status": info.status}
    del G, X
    for m, guard in ((16, 0), (64, 3)):
        G = SMG(shape, c, 1, 0, max_nrhs=m + guard)
        X0 = torch.from_numpy(synth.block(n ** 3, m + guard, 3)).to(dev)
        G.lobpcg(X0, rtol=1e-8, max_iter=2, guard=guard)          # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam, X, info = G.lobpcg(X0, rtol=1e-8, max_iter=400, guard=guard)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ex = smallest_eigs(n, c[0], m)
        res[f"lobpcg_128_m{m}"] = {
            "s": dt, "iters": info.iters, "nconv": info.nconv, "guard": guard, "status": info.status,
            "max_rel_eig_err_vs_closed_form": float(np.max(np.abs(lam[:m] - ex) / ex)),
            "max_resnorm": float(info.resnorms[:m].max())}
        # the Gram product of the full basis [X, W, P] (k = 3(m + guard)) on the FP64 matrix cores;
        # algorithmic flops of the symmetric product: 2 N per distinct entry, k (k + 1) / 2 entries
        k = 3 * (m + guard)
        gms = G.profile_gram(m + guard, k, reps=5)
        tf = float(n ** 3) * k * (k + 1) / (gms * 1e-3) / 1e12
        # the product reads the N x k basis once (8 N k bytes) for N k (k+1)
        # flops: (k+1)/8 flop per byte against the machine balance 78.6 TFLOP/s
        # / 8 TB/s, so narrow bases are bound by HBM and wide ones by the MFMAs
        gbs = 8.0 * float(n ** 3) * k / (gms * 1e-3) / 1e9
        bound = "hbm" if (k + 1) / 8.0 < 78.6e12 / (HBM_PEAK_GBS * 1e9) else "mfma"
        res[f"lobpcg_128_m{m}"]["gram"] = {"k": k, "ms": gms, "tflops": tf, "peak_tflops": 78.6,
                                           "mfma_frac": tf / 78.6, "hbm_gbs": gbs,
                                           "hbm_frac": gbs / HBM_PEAK_GBS, "bound": bound,
                                           "frac": gbs / HBM_PEAK_GBS if bound == "hbm" else tf / 78.6,
                                           "flops": "N k (k+1) (symmetric)", "bytes": "8 N k"}
        del G, X
        torch.cuda.empty_cache()
    return res


def batch_config(torch, dev):
    """48 independent FPCG-SMG(1,0) solves on boxes with nx, ny, nz drawn from
    32..96 (unit grid size, b ~ U[-1,1) seeds 1000 + box): one batched solve
    (grouped launches, graph-replayed iteration) against the 48 solves one
    after another, with every box checked bitwise against its own solve."""
    import synth
    from paper_1212_6680_amd.smg import SMG, SMGBatch
    dims = synth.box_dims(48, 32, 96, 4)
    Gs = [SMG(d, (1.0, 1.0, 1.0), 1, 0) for d in dims]
    bs = [torch.from_numpy(synth.rhs(*d, 1000 + i)).to(dev) for i, d in enumerate(dims)]
    for G, b in zip(Gs, bs):
        G.fpcg(b, max_iter=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    singles = [G.fpcg(b) for G, b in zip(Gs, bs)]
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    xs = [torch.empty_like(b) for b in bs]
    t0 = time.perf_counter()
    B = SMGBatch(Gs, bs, xs, use_graph=True)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    B.fpcg(max_iter=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = B.fpcg()
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    steps, launches = B.stats()
    same = all(torch.equal(x, xr) and i.iters == ir.iters for x, i, (xr, ir) in zip(xs, infos, singles))
    return {"boxes": 48, "dof": int(sum(G.n for G in Gs)), "s": t_batch, "sequential_s": t_seq,
            "speedup": t_seq / t_batch, "create_s": t_create,
            "grouped_launches_per_iteration": steps, "box_launches_per_iteration": launches,
            "iters_min": min(i.iters for i in infos), "iters_max": max(i.iters for i in infos),
            "all_converged": all(i.status == 0 for i in infos), "bitwise_equal_to_single_solves": bool(same)}


def varcoef_config(torch, dev, n=256, kind="aniso_layers"):
    """Variable coefficients at n^3 (unit cube): -div(kappa grad u) with z-layers
    of 2..9 planes whose conductivity alternates between 1 and 1000, and 100:1
    in-plane anisotropy in every other layer (synth.conductivity), b ~ U[-1,1)
    seed 7.  FPCG to 1e-8 with SMG (1,0) and (1,1), operator-dependent and
    linear interpolation; setup and V-cycle times."""
    import synth
    from paper_1212_6680_amd.smg import SMG
    shape = (n, n, n)
    c = ((n + 1.0) ** 2,) * 3
    coef = [torch.from_numpy(a).to(dev) for a in synth.diffusion_stencil(shape, *synth.conductivity(shape, kind, 11), c=c)]
    b = torch.from_numpy(synth.rhs(n, n, n, 7)).to(dev)
    out = {"grid": n, "field": kind, "contrast": 1e3, "anisotropy": 100.0}
    for interp in ("operator", "linear"):
        for pp in ((1, 0), (1, 1)):
            if interp == "linear" and pp == (1, 1):
                continue
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            G = SMG.variable(shape, *coef, *pp, interp=interp)
            torch.cuda.synchronize()
            setup = time.perf_counter() - t0
            x = torch.empty_like(b)
            G.fpcg(b, x, max_iter=3, zero_x0=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = G.fpcg(b, x, zero_x0=True)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            s = torch.empty_like(b)
            G.apply(b, s)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(5):
                G.apply(b, s)
            torch.cuda.synchronize()
            vc = (time.perf_counter() - t1) / 5
            out[f"fpcg_{pp[0]}{pp[1]}_{interp}"] = {"s": dt, "iters": info.iters, "status": info.status,
                                                    "true_rel_res": info.true_rel_res, "setup_s": setup,
                                                    "vcycle_ms": 1e3 * vc, "vcycle_gdof_per_s": n ** 3 / vc / 1e9}
            del G
            torch.cuda.empty_cache()
    return out


def learned_config(torch, dev, npairs=2000, steps=2000):
    """Learned post-smoother: trained at 128^3 on 2000 (r', e') pairs from
    SMG(1,0) (b seeds 10000 + i, energy-norm loss, one Adam step per pair),
    then used inside FPCG at 256^3 (b seed 6) beside SMG (1,0) and (1,1)."""
    import synth
    from paper_1212_6680_amd.smg import SMG, Net
    n = 128
    shape, c = (n, n, n), ((n + 1.0) ** 2,) * 3
    Gp, Ge = SMG(shape, c, 1, 0), SMG(shape, c, 1, 1)
    net = Net(n ** 3, "bf16", train=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    inputs, targets, _ = net.make_pairs(Gp, Ge, npairs, 10000, exact_rtol=1e-10)
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    net.set_params(synth.he_init(0))
    order = np.resize(np.random.default_rng(0).permutation(npairs), steps)
    lr = 2e-3 * (0.05 + 0.95 * 0.5 * (1 + np.cos(np.pi * np.arange(steps) / steps)))
    t0 = time.perf_counter()
    hist = net.train(shape, inputs, targets, order, lr, loss="energy")
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    params = net.get_params()
    del inputs, targets, net, Gp, Ge
    torch.cuda.empty_cache()
    n = 256
    shape, c = (n, n, n), ((n + 1.0) ** 2,) * 3
    b = torch.from_numpy(synth.rhs(n, n, n, 6)).to(dev)
    G10, G11 = SMG(shape, c, 1, 0), SMG(shape, c, 1, 1)
    ev = Net(n ** 3, "bf16", train=False)
    ev.set_params(params)
    out = {"train_grid": 128, "pairs": npairs, "adam_steps": steps, "pairs_s": t_pairs, "train_s": t_train,
           "loss_first": float(hist[:10].mean()), "loss_last": float(hist[-100:].mean())}
    for name, fn in (("smg10", lambda: G10.fpcg(b)), ("smg11", lambda: G11.fpcg(b)),
                     ("learned", lambda: G10.fpcg_learned(ev, b))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = fn()
        torch.cuda.synchronize()
        out[name] = {"s": time.perf_counter() - t0, "iters": info.iters, "status": info.status,
                     "true_rel_res": info.true_rel_res}
        if name == "learned":
            out[name]["fallback_iter"] = info.fallback_iter
            out[name]["fallback_reason"] = info.fallback_reason
    return out


def host_cpu_info():
    """The host's processors as lscpu reports them, and the CPUs this process may use."""
    import subprocess
    info = {"logical_cpus": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0)),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        kv = dict((k.strip(), v.strip()) for k, v in (ln.split(":", 1) for ln in txt.splitlines() if ":" in ln))
        for key, name in (("Model name", "model"), ("Socket(s)", "sockets"), ("Core(s) per socket", "cores_per_socket"),
                          ("Thread(s) per core", "threads_per_core"), ("CPU max MHz", "max_mhz")):
            if key in kv:
                info[name] = kv[key]
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def oracle_beside(torch, dev, configs):
    """The CPU oracle timed beside the GPU on the other workloads: every
    method and smoothing at 32^3 (whole solves, both sides); FPCG-SMG(1,0) at
    384^3 in FP64 (whole solve); LOBPCG m = 16 at 128^3 on a bounded sample of
    3 iterations (the oracle's per-iteration time beside the GPU's)."""
    import synth
    from oracle import lobpcg as OL
    from oracle import oracle as O
    from paper_1212_6680_amd.smg import SMG
    res = {"threads": O.num_threads()}
    n = 32
    shape, c = (n, n, n), ((n + 1.0) ** 2,) * 3
    b = synth.rhs(n, n, n, 1)
    bd = torch.from_numpy(b).to(dev)
    c1 = {}
    for pp in ((1, 1), (1, 0)):
        S = O.SMG(shape, c, *pp)
        G = SMG(shape, c, *pp)
        for name, meth in (("pcg", O.PCG), ("fpcg", O.FPCG), ("psd", O.PSD)):
            maxit = 100 if (name == "pcg" and pp == (1, 0)) else 500
            t0 = time.perf_counter()
            ref = O.krylov(meth, b, shape, c, S, max_iter=maxit, history=False)
            t_cpu = time.perf_counter() - t0
            getattr(G, name)(bd, max_iter=3)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = getattr(G, name)(bd, max_iter=maxit)
            torch.cuda.synchronize()
            c1[f"{name}_{pp[0]}{pp[1]}"] = {"oracle_s": t_cpu, "oracle_iters": ref.iters, "gpu_s": time.perf_counter() - t0,
                                            "gpu_iters": info.iters, "status": [ref.status, info.status]}
    res["c1_32"] = c1
    n = 384
    shape, c = (n, n, n), ((n + 1.0) ** 2,) * 3
    b = synth.rhs(n, n, n, 5)
    S = O.SMG(shape, c, 1, 0)
    t0 = time.perf_counter()
    ref = O.krylov(O.FPCG, b, shape, c, S, history=False)
    g = configs.get("fpcg_384_smg_f64", {})
    res["c4_384_f64"] = {"oracle_s": time.perf_counter() - t0, "oracle_iters": ref.iters, "gpu_s": g.get("s"),
                         "gpu_iters": g.get("iters")}
    del S, ref, b
    n, m, its = 128, 16, 3
    shape, c = (n, n, n), ((n + 1.0) ** 2,) * 3
    S = O.SMG(shape, c, 1, 0)
    X0 = synth.block(n ** 3, m, 3)
    apply_A = lambda V: np.stack([O.matvec(v, shape, c) for v in V])
    apply_T = lambda V: np.stack([S.apply(v) for v in V])
    t0 = time.perf_counter()
    OL.lobpcg(apply_A, apply_T, X0, rtol=1e-8, max_iter=its)
    t_cpu = time.perf_counter() - t0
    g = configs.get("lobpcg_128_m16", {})
    res["c3a_lobpcg_128_m16"] = {"oracle_s_per_iter": t_cpu / its, "sample": f"{its} iterations (setup included)",
                                 "gpu_s_per_iter": (g["s"] / g["iters"]) if g.get("iters") else None}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-single-thread", action="store_true", help="skip the single-threaded oracle leg")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned post-smoother workload")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the LOBPCG and mixed-precision workloads reported beside the headline")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="short run for counter collection: a 512 MiB device copy, then one V-cycle")
    ap.add_argument("--only", choices=["batch", "learned", "lobpcg", "precision", "varcoef"],
                    help="run one of the other workloads alone and print its result (for profiling)")
    ap.add_argument("--learned-pairs", type=int, default=2000)
    ap.add_argument("--learned-steps", type=int, default=2000)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU z-slab decomposition is a design, not a measured path.", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1212_6680_amd.smg import SMG

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.only:
        if args.only == "batch":
            out = batch_config(torch, dev)
        elif args.only == "learned":
            out = learned_config(torch, dev, args.learned_pairs, args.learned_steps)
        elif args.only == "precision":
            out = precision_configs(torch, dev)
        elif args.only == "varcoef":
            out = varcoef_config(torch, dev)
        else:
            out = lobpcg_configs(torch, dev)
        print(json.dumps({"only": args.only, **out}))
        return
    n = args.n
    shape = (n, n, n)
    c = ((n + 1.0) ** 2,) * 3
    N = n ** 3
    b_host = synth.rhs(n, n, n, 2)
    b = torch.from_numpy(b_host).to(dev)

    if args.pmc_probe:
        # the default schedule (the counters name it), three 512 MiB copies
        # (the calibration), then one V-cycle: the dispatches after the last copy
        G = SMG(shape, c, 1, 0)
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        G.apply(b)
        torch.cuda.synchronize()
        l0, clds, mw = G.schedule()
        print(json.dumps({"pmc_probe": True, "copy_bytes_read": src.numel() * 8, "copy_bytes_written": src.numel() * 8,
                          "schedule_l0": l0, "schedule_coarse_lds": clds, "schedule_march_waves": mw}))
        return

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G = SMG(shape, c, pre=1, post=0)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    # schedule autotuning (part of setup, reported on its own)
    t0 = time.perf_counter()
    tune = G.autotune(b, reps=5)
    tune_s = time.perf_counter() - t0

    x = torch.empty(N, dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        G.fpcg(b, x, rtol=1e-8, max_iter=500, zero_x0=True)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, info = G.fpcg(b, x, rtol=1e-8, max_iter=500, zero_x0=True)
        infos.append(info)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    sec_per_solve = total / args.steps
    iters = infos[-1].iters
    assert all(i.status == 0 for i in infos), infos[-1]

    # V-cycle throughput on its own
    s = torch.empty_like(b)
    G.apply(b, s)
    torch.cuda.synchronize()
    reps = 20
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        G.apply(b, s)
    ev1.record()
    torch.cuda.synchronize()
    vcycle_ms = ev0.elapsed_time(ev1) / reps

    # per-kernel profile of one V-cycle: every launch of a family is timed with
    # dispatch-stamped HIP events on the launch stream; the dominant family
    # (largest summed time) is the roofline kernel
    fams = {}
    for fam in ("down2", "coarse2", "chain2", "up2", "chain3", "resid3", "restrict3", "prolong3",
                "line_relax", "restrict2", "prolong2", "correct3"):
        nl, ms, by = G.profile_kernel(fam, b, reps=3)
        if nl:
            fams[fam] = {"launches": nl, "ms": ms, "bytes": by, "avg_us": 1e3 * ms / nl,
                         "gbs": by / (ms * 1e-3) / 1e9}
    dom = max(fams, key=lambda f: fams[f]["ms"])
    d = fams[dom]

    # the same V-cycle summed per 3D level (z-semicoarsening keeps the odd
    # planes: nz -> nz // 2); the last row is the prolongation chain that
    # spans every level
    rows = G.profile_levels(b, reps=3)
    split = {f: G.profile_levels(b, reps=3, family=f) for f in fams}
    per_level, nzl = [], n
    for i, (nl, ms, by) in enumerate(rows):
        if nl == 0:
            continue
        last = i == len(rows) - 1
        per_level.append({"level": "chain3" if last else i, "nz": None if last else nzl, "launches": nl,
                          "ms": round(ms, 4), "mb": round(by / 1e6, 2),
                          "gbs": round(by / (ms * 1e-3) / 1e9, 1) if ms > 0 else None,
                          "ms_by_family": {f: round(split[f][i][1], 4) for f in split if split[f][i][0]}})
        nzl //= 2
    achieved = d["gbs"]
    traffic = read_traffic(dom, (tune.l0, tune.coarse_lds, tune.march_waves))

    out = {
        "metric": METRIC,
        "value": sec_per_solve,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * sec_per_solve,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"FPCG-SMG(1,0) to rel. residual 1e-8, 3D 7-point Dirichlet Laplacian "
                               f"{n}^3 unit cube (c={(n + 1) ** 2}), b~U[-1,1) seed 2, x0=0",
                   "grid": [n, n, n], "smoothing": [1, 0], "rtol": 1e-8, "solver": "fpcg"},
        "iters": iters,
        "true_rel_res": infos[-1].true_rel_res,
        "setup_s": setup_s,
        "autotune": {"s": tune_s, "candidates": tune.candidates, "l0": tune.l0, "coarse_lds": tune.coarse_lds,
                     "march_waves": tune.march_waves,
                     "default_vcycle_ms": tune.default_ms, "best_vcycle_ms": tune.best_ms},
        "vcycle_ms": vcycle_ms,
        "vcycle_gdof_per_s": N / (vcycle_ms * 1e-3) / 1e9,
        "roofline": {
            "kernel": KERNEL_NAMES[dom],
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "launches_per_vcycle": d["launches"],
            "avg_launch_us": d["avg_us"],
            "algorithmic_bytes_per_launch": d["bytes"] / d["launches"],
            "share_of_vcycle": d["ms"] / vcycle_ms,
        },
        "kernels_per_vcycle": {f: {k: round(v, 4) for k, v in fams[f].items()} for f in fams},
        "levels_per_vcycle": per_level,
    }

    if not args.no_variants:
        var = {}
        for name, pp in [("fpcg_11", (1, 1)), ("pcg_11", (1, 1)), ("psd_11", (1, 1)),
                         ("psd_10", (1, 0)), ("pcg_10", (1, 0))]:
            Gv = G if pp == (1, 0) else SMG(shape, c, *pp)
            fn = getattr(Gv, name.split("_")[0])
            fn(b, rtol=1e-8, max_iter=3)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, inf = fn(b, rtol=1e-8, max_iter=100 if name == "pcg_10" else 500)
            torch.cuda.synchronize()
            var[name] = {"s": time.perf_counter() - t0, "iters": inf.iters, "status": inf.status,
                         "rel_res": inf.rel_res}
            if Gv is not G:
                del Gv
        var["fpcg_10"] = {"s": sec_per_solve, "iters": iters, "status": 0, "rel_res": infos[-1].rel_res}
        # without a preconditioner: the cost per iteration of equation (2) against (1)
        for name in ("pcg", "fpcg"):
            fn = getattr(G, name)
            fn(b, rtol=1e-8, max_iter=3, precond="none")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, inf = fn(b, rtol=1e-30, max_iter=200, precond="none")
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            var[f"{name}_noprec_200it"] = {"s": el, "iters": inf.iters, "ms_per_iter": el / max(inf.iters, 1) * 1e3}
        out["variants"] = var

    if not args.no_configs:
        out["configs"] = other_configs(torch, dev, learned=not args.no_learned)

    if not args.no_cpu_baseline:
        from oracle import oracle as O
        S = O.SMG(shape, c, 1, 0)
        threads = O.num_threads()
        t0 = time.perf_counter()
        r = O.krylov(O.FPCG, b_host, shape, c, S, rtol=1e-8, max_iter=500, history=False)
        t_cpu = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": t_cpu, "unit": "s", "cores": threads, "kind": "oracle",
                               "sample": f"the whole FPCG-SMG(1,0) solve at {n}^3 ({r.iters} iterations, "
                                         f"setup excluded), FP64 C/OpenMP oracle",
                               "iters": r.iters, "host": host_cpu_info()}
        if not args.no_single_thread:
            O.set_num_threads(1)
            t0 = time.perf_counter()
            r1 = O.krylov(O.FPCG, b_host, shape, c, S, rtol=1e-8, max_iter=500, history=False)
            out["cpu_baseline"]["single_thread"] = {"value": time.perf_counter() - t0, "unit": "s", "cores": 1,
                                                    "iters": r1.iters}
            O.set_num_threads(threads)
        del S
        if not args.no_configs:
            out["oracle_beside"] = oracle_beside(torch, dev, out.get("configs", {}))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
