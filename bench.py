"""Benchmark of the coded-QR hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c5] [--legs fp64,fp32]

One step = the whole path on one synthetic input already resident in HBM:
place A into the encoded buffer, encode, factor with the workload's scheduled
node failures (erase + recover at the start of the scheduled panels),
post-orthogonalize Q_1 and the right-hand side.  Prints ONE JSON line.

The default workload is the largest one-GPU configuration: n = 32768
Gaussian, 16 x 16 grid, b = 256, K = 8 in-node checksums, a reverse-diagonal
storm of f_tol = 4 failures per grid line every 16 panels.  Each precision leg
(FP64; the coefficient product R_bar on FP32 MFMA) runs the same input and
schedule; `value` is the first leg's rate.

value = coded-QR TFLOP/s = model flops / step time, with the model
F = m' (4 n^2 + 4 n d + 4 n b) (right-looking update incl. carried checksum
columns, left re-projection, CGS2 panels).  Also reported per leg: the coding
overhead over the uncoded factorization (same library, K = 0) next to its
algorithmic floor (1 + c/m)(1 + d/n) - 1, recovery time per failure event,
error norms; the roofline of the dominant kernel measured with HIP events on
the library's stream; and the FP64 CPU oracle timed on the host cores.
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
sys.path.insert(0, ROOT)

import synth  # noqa: E402

PEAK = {"fp64_mfma_tflops": 78.6, "fp32_mfma_tflops": 157.3, "bf16_mfma_tflops": 2500.0, "hbm_gbs": 8000.0}

WORKLOADS = {
    # n, pr, K, b, storage, failure kind, nfail
    "c1": dict(n=256, pr=4, K=1, b=16, storage="out", kind="random", nfail=1,
               desc="n=256 Gaussian, 4x4 grid (64x64 blocks), b=16, K=1 out-of-node, 1 node failure at a random panel"),
    "c2": dict(n=4096, pr=8, K=2, b=64, storage="in", kind="random", nfail=2,
               desc="n=4096 Gaussian FP64, 8x8 grid (512x512 blocks), b=64, K=2 in-node checksums (f_tol=1), "
                    "2 random node failures at random panels"),
    "c3": dict(n=16384, pr=8, K=4, b=128, storage="out", kind="revdiag", nfail=4, cpu_sample_n=4096,
               desc="n=16384 Gaussian FP64, 8x8 grid (2048x2048 blocks), b=128, K=4 out-of-node (f_tol=4), "
                    "reverse-diagonal failures every 16 panels"),
    "c5": dict(n=32768, pr=16, K=8, b=256, storage="in", kind="revdiag", nfail=4, cpu_sample_n=8192,
               desc="n=32768 Gaussian FP64, 16x16 grid (2048x2048 blocks), b=256, K=8 in-node (f_tol=4), "
                    "reverse-diagonal failures every 16 panels"),
}


# Phases whose kernel is bound by FP64 MFMA throughput (products with one
# 64-wide dimension and a long reduction: 16 flop per byte, above the
# 78.6 TFLOP/s / 8 TB/s ridge); the rest are bound by HBM bytes.
MFMA_PHASES = {"reproj_product", "reproj_update", "panel_gram", "inpanel_projection", "trailing_product"}
SINGLE_KERNEL_PHASES = ("trailing_product", "trailing_update", "reproj_product", "panel_gram", "recover",
                        "postorth")
KERNEL_OF = {
    "encode": "encode_fused_kernel / encode_rows_kernel",
    "reproj_product": "tn_lds_kernel<1, false>", "reproj_update": "nn_kernel<*, 1>",
    "panel_gram": "tn_lds_kernel<2, false>", "panel_chol": "chol_kernel", "panel_transform": "apply_kernel / nn1_apply_kernel",
    "inpanel_projection": "tn/nn <2, false>",
    "trailing_product": "tn_lds_kernel<0, false>", "trailing_update": "nnw_kernel<0>",
    "split_reduce": "tn_reduce_kernel / nn_reduce_kernel", "recover": "line_kernel",
    "postorth": "postorth_kernel", "erase": "erase_kernel", "other": "zero_ints_kernel / fill_zero_kernel",
    "solve": "trinv_kernel / gemv_t_kernel / trsv_step_kernel",
}


def model_flops(mp, n, d, b, reproject=True):
    """Flops of the coded blocked Gram-Schmidt: right-looking update 2 m' n^2,
    carried checksum columns 4 m' n d, CGS2 panels 4 m' n b, and the left
    re-projection 2 m' n^2 when it runs."""
    return mp * ((4.0 if reproject else 2.0) * n * n + 4.0 * n * d + 4.0 * n * b)


def workload_inputs(name: str, ftol: int, seed: int = 0) -> dict:
    """Seeded inputs of a workload: A, the right-hand side, the generator draws
    and the failure schedule (shared with the full-size parity test).  ftol is
    the code's failure tolerance per grid line (sizes reverse-diagonal storms)."""
    w = WORKLOADS[name]
    n, pr, K, b = w["n"], w["pr"], w["K"], w["b"]
    return {
        "A": synth.gaussian(n, n, seed),
        "rhs": synth.gaussian(n, 1, seed + 1),
        "v": synth.q_generator_draws(K, pr, seed),
        "gh": synth.r_generator_draws(pr, K, seed),
        # "random": nfail single-node events at independent random panels
        # (events sharing a panel hit distinct grid rows and columns)
        "schedule": synth.draw_schedule(w["kind"], n // b, pr, pr, seed, nfail=w["nfail"], every=16, f=ftol),
    }


def conditioned_input(n: int, cond: float, seed: int, dev) -> np.ndarray:
    """A = U diag(s) V^T with Haar U, V (sign-fixed QR of seeded Gaussians) and
    s_i = cond^(-i/(n-1)).  Small sizes use the shared numpy generator; large
    ones run the QRs on the device (input generation only, outside timing)."""
    if n <= 4096:
        return synth.conditioned(n, cond, seed)
    import torch
    g = torch.Generator().manual_seed(seed)

    def haar():
        z = torch.randn(n, n, generator=g, dtype=torch.float64).to(dev)
        qm, rm = torch.linalg.qr(z)
        return qm * torch.sign(torch.diagonal(rm))

    u, v = haar(), haar()
    s = cond ** (-torch.arange(n, dtype=torch.float64, device=dev) / max(n - 1, 1))
    a = (u * s) @ v.T
    out = np.asfortranarray(a.cpu().numpy())
    del u, v, a
    torch.cuda.empty_cache()
    return out


def kernel_source_hash(kernel: str) -> str:
    """Hash of one kernel's definition (from its template line to its closing
    brace) in the library's sources, e.g. kernel = "nnq_kernel<0>"; "" if not
    found.  A traffic record holds for the kernel text it was measured on."""
    name = kernel.split("<")[0]
    csrc = os.path.join(ROOT, "paper_2311_11943_amd", "csrc")
    for src in sorted(os.listdir(csrc)):
        if not src.endswith((".hip", ".hpp", ".cpp")):
            continue
        with open(os.path.join(csrc, src)) as f:
            lines = f.read().split("\n")
        for i, line in enumerate(lines):
            if f"void {name}(" in line and "__global__" in line:
                start = i - 1 if i > 0 and lines[i - 1].startswith("template") else i
                end = next(j for j in range(i, len(lines)) if lines[j] == "}")
                return hashlib.sha256("\n".join(lines[start:end + 1]).encode()).hexdigest()[:16]
    return ""


def traffic_record(phase: str, workload: str):
    """HBM traffic per launch measured by rocprofv3 counters (profiles/), only
    if it was taken on the current text of that kernel."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    key = f"{workload}:{phase}"
    r = rec.get(key)
    if not r or r.get("source_hash") != kernel_source_hash(r.get("kernel", "")):
        return None
    return r.get("bytes_per_launch")


def run_sweep(args):
    """The paper's overhead experiments on one GPU (T_coding vs p and vs f;
    T_enc and p T_recov vs f): n = 24000 Gaussian, p = p_r = p_c in
    {6, 8, 10, 12}, f = K out-of-node checksums in {0, 1, 2, 3}, one panel per
    grid block column (b = n/p, factored recursively in leaves of <= 64
    columns), a reverse-diagonal failure of f nodes per grid row and column at
    every panel boundary.  One JSON line per (p, f)."""
    import torch
    from paper_2311_11943_amd import cqr
    dev = torch.device("cuda:0")
    n = args.sweep_n
    A_host = synth.gaussian(n, n, args.seed)
    A = cqr.to_device_colmajor(A_host, dev)
    del A_host

    def ev_ms(fn):
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        z.record()
        torch.cuda.synchronize()
        return a.elapsed_time(z)

    for p in (6, 8, 10, 12):
        b = n // p
        # uncoded factorization time (same library, no checksums)
        qu = cqr.CodedQR(cqr.Config(n, n, p, p, 0, 0, b, cqr.CQR_OUT_OF_NODE), None, None, dev)
        Au, Ru = qu.alloc()
        t_qr = []
        for _ in range(2):
            Au.copy_(A)
            t_qr.append(ev_ms(lambda: qu.factor(Au, Ru)))
        T_qr = t_qr[-1]
        qu.close()
        del Au, Ru
        for f in (0, 1, 2, 3):
            if f == 0:
                print(json.dumps({"sweep": "coding overhead vs p and f", "n": n, "p": p, "f": 0, "b": b,
                                  "T_QR_ms": round(T_qr, 3)}), flush=True)
                continue
            cfg = cqr.Config(n, n, p, p, f, f, b, cqr.CQR_OUT_OF_NODE)
            q = cqr.CodedQR(cfg, synth.q_generator_draws(f, p, args.seed), synth.r_generator_draws(p, f, args.seed),
                            dev)
            At, R = q.alloc()
            Qpost = cqr.col_major(n, n, dev)

            def enc():
                At[:n, :n].copy_(A)
                q.encode(At)
            enc()
            t_copy = ev_ms(lambda: At[:n, :n].copy_(A))
            T_enc = ev_ms(enc) - t_copy
            T_fac = ev_ms(lambda: q.factor(At, R))
            T_post = ev_ms(lambda: q.postorth(At, Qpost))
            # the same factorization with a reverse-diagonal failure at every panel boundary
            sched = synth.draw_schedule("revdiag", p, p, p, args.seed, every=1, f=f)
            enc()
            k, t_rec = 0, 0.0
            for t, nodes in sched:
                q.factor(At, R, k, t)
                k = t
                q.erase(At, R, nodes)
                t_rec += ev_ms(lambda: q.recover(At, R, nodes))
            q.factor(At, R, k, cfg.npanels)
            torch.cuda.synchronize()
            res = (torch.linalg.norm(A - At[:n, :n] @ R[:, :n]) / torch.linalg.norm(A)).item()
            Qt = At[:, :n]
            orth = torch.linalg.norm(torch.eye(n, device=dev, dtype=torch.float64) - Qt.T @ Qt).item()
            T_rec = t_rec / max(len(sched), 1)
            print(json.dumps({
                "sweep": "coding overhead vs p and f", "n": n, "p": p, "f": f, "b": b,
                "T_QR_ms": round(T_qr, 3), "T_enc_ms": round(T_enc, 3), "T_factor_coded_ms": round(T_fac, 3),
                "T_post_ms": round(T_post, 3),
                "T_coding_pct": round(100 * (T_enc + T_fac + T_post - T_qr) / T_qr, 2),
                "floor_pct": round(100 * ((1 + f / p) ** 2 - 1), 2),
                "T_recov_ms_per_event": round(T_rec, 3), "p_T_recov_ms": round(p * T_rec, 3),
                "events": len(sched), "nodes_per_event": len(sched[0][1]) if sched else 0,
                "errors_with_failures": {"residual": res, "orth_coded": orth, "info": q.info()},
            }), flush=True)
            q.close()
            del At, R, Qpost, Qt
            torch.cuda.empty_cache()


def run_peaks(args):
    """Practical ceilings of this device beside the published peaks used for
    the rooflines: a large square GEMM in FP64 and FP32 through torch (the
    vendor BLAS, MFMA) and a device-to-device copy (HBM read + write)."""
    import torch
    dev = torch.device("cuda:0")

    def best_ms(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            z.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(z))
        return min(ts)

    out = {"peaks": "measured ceilings vs published", "device": torch.cuda.get_device_name(0)}
    n = 8192
    for name, dt in (("fp64", torch.float64), ("fp32", torch.float32)):
        x = torch.randn(n, n, device=dev, dtype=dt)
        y = torch.randn(n, n, device=dev, dtype=dt)
        zz = torch.empty(n, n, device=dev, dtype=dt)
        ms = best_ms(lambda: torch.matmul(x, y, out=zz))
        out[f"gemm_{name}_tflops"] = round(2.0 * n ** 3 / (ms * 1e-3) / 1e12, 2)
        del x, y, zz
    out["published_fp64_mfma_tflops"] = PEAK["fp64_mfma_tflops"]
    out["published_fp32_mfma_tflops"] = PEAK["fp32_mfma_tflops"]
    src = torch.ones(256 << 20, device=dev, dtype=torch.float64)   # 2 GiB
    dst = torch.empty_like(src)
    ms = best_ms(lambda: dst.copy_(src))
    out["copy_gbs"] = round(2.0 * src.numel() * 8 / (ms * 1e-3) / 1e9, 1)
    out["published_hbm_gbs"] = PEAK["hbm_gbs"]
    print(json.dumps(out), flush=True)


def run_adjoint(args):
    """Least squares through the coded QR and its adjoint, on the tall-skinny
    workload (c4: m = 65536, n = 512 Gaussian A and b, 16 x 1 grid of 4096-row
    blocks, b = 64, K_v = 2 out-of-node checksum block rows, no horizontal
    code, two nodes failing at once at a random panel) or on the n = 32768
    workload (c5: its grid, code and failure storms).
    loss = ||x - x_t||^2 with x = R_1^{-1} (G_0 Q_1)^T (G_0 b); the forward
    (encode, factor, post-orthogonalization, solve) and the backward
    (coded_qr_solve_backward, coded_qr_backward) are timed separately, and the
    gradient is checked against the closed form of the W-weighted least squares
    (W = I + G_v^T G_v; for square A the exact solve).  One JSON line."""
    import torch
    from paper_2311_11943_amd import autograd as ag
    from paper_2311_11943_amd import cqr
    dev = torch.device("cuda:0")
    prec = PRECISIONS[args.precision]["code"]
    if args.adjoint_workload == "c5":
        w = WORKLOADS["c5"]
        m = n = w["n"]
        pr, K, b = w["pr"], w["K"], w["b"]
        cfg = cqr.Config(m, n, pr, pr, K, K, b, cqr.CQR_IN_NODE, precision=prec)
        engine = cqr.CodedQR(cfg, synth.q_generator_draws(K, pr, args.seed), synth.r_generator_draws(pr, K, args.seed),
                             dev)
        sched = synth.draw_schedule(w["kind"], n // b, pr, pr, args.seed, nfail=w["nfail"], every=16, f=engine.ftol)
        desc = "c5: " + w["desc"]
        grid = f"{pr}x{pr}"
    else:
        m, n, pr, K, b = 65536, 512, 16, 2, 64
        cfg = cqr.Config(m, n, pr, 1, K, 0, b, cqr.CQR_OUT_OF_NODE, precision=prec)
        # two nodes fail at once at a random panel (R is protected by its checksum rows)
        sched = synth.draw_schedule("burst", n // b, pr, 1, args.seed, nfail=2)
        engine = cqr.CodedQR(cfg, synth.q_generator_draws(K, pr, args.seed), None, dev)
        desc = ("c4: m=65536, n=512 Gaussian A and b, 16x1 grid (4096-row blocks), b=64, K_v=2 out-of-node, no "
                "horizontal code (R protected by its checksum rows), 2 nodes failing at once at a random panel")
        grid = "16x1"
    A = torch.tensor(synth.gaussian(m, n, args.seed), device=dev, requires_grad=True)
    B = torch.tensor(synth.gaussian(m, 1, args.seed + 1), device=dev, requires_grad=True)
    xt = torch.tensor(synth.gaussian(n, 1, args.seed + 2), device=dev)

    def fwd():
        Q, R1 = ag.coded_qr(A, engine, sched, recompute=args.recompute)
        return ag.coded_solve(Q, R1, B, engine)

    def ev():
        return torch.cuda.Event(enable_timing=True)

    f_ms, b_ms = [], []
    for it in range(args.warmup + args.steps):
        A.grad = None
        B.grad = None
        e0, e1, e2 = ev(), ev(), ev()
        e0.record()
        x = fwd()
        loss = ((x - xt) ** 2).sum()
        e1.record()
        loss.backward()
        e2.record()
        torch.cuda.synchronize()
        if it >= args.warmup:
            f_ms.append(e0.elapsed_time(e1))
            b_ms.append(e1.elapsed_time(e2))
        print(f"[bench] adjoint step {it + 1} of {args.warmup + args.steps}: forward {e0.elapsed_time(e1):.1f} ms, "
              f"backward {e1.elapsed_time(e2):.1f} ms", file=sys.stderr, flush=True)
    fm, bm = sum(f_ms) / len(f_ms), sum(b_ms) / len(b_ms)
    # closed form: W v = v + G_v^T (G_v v), with G_v = G~_v (x) I_bs
    gv = torch.tensor(engine.generators()[0], device=dev)

    def W(vm):
        vm = vm.detach()
        blocks = vm.reshape(pr, -1)                  # block t of rows in row t
        chk = gv @ blocks                            # G_v v, one row per checksum block
        return vm + (gv.T @ chk).reshape(m, -1)

    Ad, Bd = A.detach(), B.detach()
    gA, gB = A.grad, B.grad
    del A, B
    if m == n:
        # square A: x = A^{-1} b whatever W is; db = A^{-T} g, dA = -db x^T (g = 2 (x - x_t)),
        # from LU solves with A itself (the normal equations would square its condition number)
        xw = torch.linalg.solve(Ad, Bd)
        cB = torch.linalg.solve(Ad.T, 2 * (xw - xt))
        cA = -cB @ xw.T
    else:
        WA = W(Ad)
        H = Ad.T @ WA
        xw = torch.linalg.solve(H, WA.T @ Bd)
        z = torch.linalg.solve(H, 2 * (xw - xt))
        del H
        cB = WA @ z
        cA = W(Bd - Ad @ xw) @ z.T
        cA -= WA @ z @ xw.T
        del WA
    print("[bench] closed-form gradient done", file=sys.stderr, flush=True)
    relA = ((gA - cA).abs().max() / cA.abs().max()).item()
    relB = ((gB - cB).abs().max() / cB.abs().max()).item()
    relx = ((x.detach() - xw).abs().max() / xw.abs().max()).item()
    mp = cfg.mp
    f_fl = model_flops(mp, n, cfg.N - n, b) + 2.0 * m * n + n * n
    b_fl = 6.0 * mp * n * n + 2.0 * n ** 3
    print(json.dumps({
        "metric": "coded-QR least-squares forward + adjoint time", "value": round(fm + bm, 4), "unit": "ms",
        "higher_is_better": False, "steps": args.steps, "warmup": args.warmup,
        "dtype": PRECISIONS[args.precision]["dtype"] + ("" if args.precision == "fp64" else " (adjoint f64)"),
        "data": "synthetic",
        "config": {"workload": desc, "m": m, "n": n, "grid": grid, "b": b, "K": K, "precision": args.precision,
                   "recompute": args.recompute,
                   "failure_schedule": [[t, [list(x) for x in nodes]] for t, nodes in sched]},
        "forward_ms": round(fm, 4), "backward_ms": round(bm, 4),
        "forward_tflops": round(f_fl / (fm * 1e-3) / 1e12, 3), "backward_tflops": round(b_fl / (bm * 1e-3) / 1e12, 3),
        "errors": {"x_vs_weighted_ls": relx, "dA_vs_closed_form": relA, "db_vs_closed_form": relB},
    }), flush=True)
    engine.close()


def _submatrix_extremes(task):
    """Smallest |det| and largest 2-norm condition number over the k x k
    submatrices of G with row set `rows` and column sets starting at column c0."""
    import itertools
    G, k, rows, c0 = task
    p = G.shape[1]
    mind, maxc = np.inf, 0.0
    rest = itertools.combinations(range(c0 + 1, p), k - 1)
    while True:
        chunk = list(itertools.islice(rest, 200000))
        if not chunk and k > 1:
            break
        cols = np.array([(c0,) + c for c in chunk], dtype=np.int64) if k > 1 else np.array([[c0]])
        sub = G[np.ix_(rows, range(p))][:, cols].transpose(1, 0, 2)      # (N, k, k)
        mind = min(mind, float(np.abs(np.linalg.det(sub)).min()))
        sv = np.linalg.svd(sub, compute_uv=False)
        maxc = max(maxc, float((sv[:, 0] / sv[:, -1]).max()))
        if k == 1:
            break
    return mind, maxc


def run_generator_study(args):
    """The paper's check of its Q-side generator (the experiment behind its
    figure comparing structured and random generators): smallest |det| and
    largest condition number over all square submatrices of the structured
    G~ = [G~_1  V~] (G~_1 = -1/2 V~ V~^T; checked against the library's plan
    generator wherever a plan can hold the grid) and of the
    completely random G~' = [G~_1'  V~] (G~_1' i.i.d. Unif(0, 1), same V~), for
    f = 2..6 checksum rows and p_r = 16, 32, 64 grid rows, averaged (in log10)
    over trials.  Host only, one JSON line per (p_r, f)."""
    import itertools
    import multiprocessing as mp
    from paper_2311_11943_amd import cqr
    # the paper's protocol: 100 trials, 10 for the largest case (about 1.5 h on
    # six host processes; --study-scale shortens it)
    trials = {(pr, f): 100 for pr in (16, 32, 64) for f in range(2, 7)}
    trials[(64, 6)] = 10
    scale = args.study_scale
    with mp.Pool(args.study_procs) as pool:
        for pr in (16, 32, 64):
            for f in range(2, 7):
                nt = max(1, int(round(trials[(pr, f)] * scale)))
                logs = {"structured": [], "random": []}
                t0 = time.perf_counter()
                for t in range(nt):
                    v = synth.q_generator_draws(f, pr, 1000 + t)
                    # the construction's definition; the library's plans hold at most 32 blocks per code
                    # line, so where one can be made its generator must agree with this one
                    gv = np.hstack([-0.5 * v @ v.T, v])
                    if pr + f <= 32:
                        cfg = cqr.Config(m=16 * pr, n=16 * pr, pr=pr, pc=1, kv=f, kh=0, b=16)
                        plan = cqr.coded_qr_plan_create(cfg, v, None)
                        glib, _ = cqr.coded_qr_plan_generators(plan, cfg)
                        cqr.coded_qr_plan_destroy(plan)
                        assert np.abs(glib - gv).max() <= 1e-14 * np.abs(gv).max()
                    rng = np.random.default_rng(5000 + t)
                    gr = gv.copy()
                    gr[:, :f] = rng.uniform(0.0, 1.0, (f, f))
                    for name, G in (("structured", gv), ("random", gr)):
                        tasks = [(G, k, list(rows), c0) for k in range(1, f + 1)
                                 for rows in itertools.combinations(range(f), k) for c0 in range(pr - k + 1)]
                        res = pool.map(_submatrix_extremes, tasks, chunksize=4)
                        logs[name].append((np.log10(min(r[0] for r in res)), np.log10(max(r[1] for r in res))))
                out = {"study": "generator submatrix conditioning", "p_r": pr, "f": f, "trials": nt,
                       "seconds": round(time.perf_counter() - t0, 1)}
                for name, vals in logs.items():
                    a = np.array(vals)
                    out[name] = {"log10_min_abs_det": round(float(a[:, 0].mean()), 3),
                                 "log10_max_cond": round(float(a[:, 1].mean()), 3)}
                out["max_cond_ratio_structured_over_random"] = round(
                    10 ** (out["structured"]["log10_max_cond"] - out["random"]["log10_max_cond"]), 3)
                print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS))
    ap.add_argument("--legs", default="fp64,fp32,bf16x3",
                    help="comma-separated precision legs timed on the same input and schedule; the first gives "
                         "`value` (fp64: FP64 throughout; fp32: the coefficient product R_bar on FP32 MFMA)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip overhead/profile/oracle legs")
    ap.add_argument("--skip-uncoded", action="store_true",
                    help="skip the uncoded leg (so that a kernel trace of the command holds only the coded "
                         "factorization's launches, the ones the roofline averages)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the run, launch one plain copy kernel of 512 MiB (y = 2x) as the reference for "
                         "HBM byte counters")
    ap.add_argument("--precision", default="fp64", choices=tuple(PRECISIONS),
                    help="--adjoint only: the forward's coefficient products in this precision (the adjoint is FP64)")
    ap.add_argument("--cond", type=float, default=0.0,
                    help="> 0: A = U diag(s) V^T with Haar U, V and log-spaced s of this condition number "
                         "instead of a Gaussian A")
    ap.add_argument("--lookahead", type=int, default=1, choices=(0, 1),
                    help="1: overlap the next panel with the trailing update on a second stream")
    ap.add_argument("--panel", default="cholqr2", choices=("cholqr2", "cgs2", "icgs", "mgs"),
                    help="panel method (cholqr2: two Cholesky-QR passes; the others column-wise)")
    ap.add_argument("--no-reproject", action="store_true",
                    help="the paper's blocked Gram-Schmidt without the left re-projection of each panel")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the benchmark line: the paper's coding-overhead grid (n = 24000, "
                         "p in {6, 8, 10, 12}, f in {0..3}), one JSON line per point")
    ap.add_argument("--sweep-n", type=int, default=24000)
    ap.add_argument("--adjoint", action="store_true",
                    help="instead of the benchmark line: forward + adjoint of a least-squares loss through the coded "
                         "QR and the coded solve, one JSON line")
    ap.add_argument("--recompute", action="store_true",
                    help="--adjoint: keep only A for the backward and factor again there")
    ap.add_argument("--adjoint-workload", default="c4", choices=("c4", "c5"),
                    help="--adjoint: c4 (m = 65536, n = 512, 16 x 1 grid) or c5 (n = 32768, 16 x 16 grid)")
    ap.add_argument("--reps", type=int, default=0,
                    help="repetitions of each timed extra (overhead legs); 0: 2 from n = 16384 on, else 5")
    ap.add_argument("--generator-study", action="store_true",
                    help="host only: smallest |det| and largest condition number over all square submatrices of "
                         "the structured and of a random Q-side generator (f = 2..6, p_r = 16, 32, 64)")
    ap.add_argument("--study-scale", type=float, default=1.0, help="scales the study's trial counts")
    ap.add_argument("--study-procs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="limit the oracle's BLAS threads in the cpu_baseline leg (0: all host threads)")
    ap.add_argument("--peaks", action="store_true",
                    help="measure the device's practical ceilings beside the published peaks: FP64 and FP32 "
                         "GEMM through torch (the vendor BLAS) and a device copy; one JSON line")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the coded-QR hot path here runs on a single MI355X "
              "(the processor grid is simulated as blocks of one matrix); --gpus must be 1.", file=sys.stderr)
        sys.exit(2)

    if args.generator_study:
        run_generator_study(args)
        return
    if args.sweep:
        run_sweep(args)
        return
    if args.adjoint:
        run_adjoint(args)
        return
    if args.peaks:
        run_peaks(args)
        return

    import torch
    from paper_2311_11943_amd import cqr

    dev = torch.device("cuda:0")
    w = WORKLOADS[args.workload]
    n, pr, K, b = w["n"], w["pr"], w["K"], w["b"]
    storage = cqr.CQR_IN_NODE if w["storage"] == "in" else cqr.CQR_OUT_OF_NODE
    legs = [x for x in args.legs.split(",") if x]
    if not legs or any(x not in PRECISIONS for x in legs):
        raise SystemExit(f"--legs takes a comma-separated list of {sorted(PRECISIONS)}")
    v = synth.q_generator_draws(K, pr, args.seed)
    gh = synth.r_generator_draws(pr, K, args.seed)
    panel = {"cholqr2": cqr.CQR_PANEL_CHOLQR2, "cgs2": cqr.CQR_PANEL_CGS2, "icgs": cqr.CQR_PANEL_ICGS,
             "mgs": cqr.CQR_PANEL_MGS}[args.panel]
    reproject = 0 if args.no_reproject else 1
    cfg0 = cqr.Config(n, n, pr, pr, K, K, b, storage, lookahead=args.lookahead)
    q0 = cqr.CodedQR(cfg0, v, gh, dev)
    ftol = q0.ftol
    q0.close()
    inp = workload_inputs(args.workload, ftol, args.seed)
    A_host, rhs_host, sched = inp["A"], inp["rhs"], inp["schedule"]
    if args.cond > 0:
        A_host = conditioned_input(n, args.cond, args.seed, dev)
    A = cqr.to_device_colmajor(A_host, dev)
    B = cqr.to_device_colmajor(rhs_host, dev)
    mp, d = cfg0.mp, cfg0.N - n
    F = model_flops(mp, n, d, b, reproject == 1)
    F_unc = model_flops(n, n, 0, b, reproject == 1)
    floor = (1 + (mp - n) / n) * (1 + d / n) - 1

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    log(f"workload {args.workload}: inputs resident, legs {legs}")
    reps = args.reps if args.reps > 0 else (2 if n >= 16384 else 5)
    out = {
        "metric": "coded-QR TFLOP/s + overhead vs uncoded; mixed vs FP64 at stated ||I-Q^TQ||",
        "value": None,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": PRECISIONS[legs[0]]["dtype"],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {w['desc']}", "n": n, "grid": f"{pr}x{pr}", "b": b,
                   "K": K, "f_tol": ftol, "storage": w["storage"],
                   "panel": {"cholqr2": "CholQR2 (block CGS2)", "cgs2": "column-wise CGS2", "icgs": "column-wise ICGS",
                             "mgs": "column-wise MGS"}[args.panel] + ("" if reproject else ", no re-projection")
                            + (" + re-projection" if reproject else ""),
                   "lookahead": args.lookahead, "legs": legs,
                   "input": "gaussian" if args.cond <= 0 else f"U diag(s) V^T, cond {args.cond:g}",
                   "failure_schedule": [[t, [list(x) for x in nodes]] for t, nodes in sched],
                   "model_flops": F, "uncoded_model_flops": F_unc},
        "legs": {},
    }
    first = None        # Q~ and R of the first leg, to compare the other legs with
    At = R = Qpost = Bpost = None
    for li, leg in enumerate(legs):
        cfg = cqr.Config(n, n, pr, pr, K, K, b, storage, reproject=reproject, lookahead=args.lookahead,
                         precision=PRECISIONS[leg]["code"], panel=panel)
        q = cqr.CodedQR(cfg, v, gh, dev)
        if At is None:
            At, R = q.alloc()
            Qpost = cqr.col_major(n, n, dev)
            Bpost = cqr.col_major(n, 1, dev)

        def step():
            At[:n, :n].copy_(A)
            q.encode(At)
            k = 0
            for t, nodes in list(sched) + [(cfg.npanels, None)]:
                q.factor(At, R, k, t)
                k = t
                if nodes is None:
                    break
                q.erase(At, R, nodes)
                q.recover(At, R, nodes)
            q.postorth(At, Qpost, B, Bpost)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        log(f"[{leg}] {args.warmup} warmup steps done")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(args.steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1) / args.steps
        log(f"[{leg}] {args.steps} timed steps done: {ms:.3f} ms per step")
        L = {"ms_per_step": round(ms, 4), "tflops": round(F / (ms * 1e-3) / 1e12, 4),
             "useful_tflops": round(F_unc / (ms * 1e-3) / 1e12, 4),
             "wall_s_timed": round(wall, 3), "arithmetic": PRECISIONS[leg]["desc"]}
        # errors of the last step (verification, outside the timed region)
        Qt = At[:, :n]
        eye = torch.eye(n, device=dev, dtype=torch.float64)
        L["errors"] = {
            "residual": (torch.linalg.norm(A - At[:n, :n] @ R[:, :n]) / torch.linalg.norm(A)).item(),
            "orth_coded": torch.linalg.norm(eye - Qt.T @ Qt).item(),
            "orth_post": torch.linalg.norm(eye - Qpost.T @ Qpost).item(),
            "info": q.info()}
        del eye
        if first is None:
            first = (At[:, :n].clone(), R.clone())
        else:
            # against the first (FP64) leg on the same input and schedule; the
            # FP64 leg matches the FP64 oracle in the parity tests
            L["vs_" + legs[0] + "_leg"] = {
                "R_max_rel": ((R - first[1]).abs().max() / first[1].abs().max()).item(),
                "Q_max_abs": (At[:, :n] - first[0]).abs().max().item()}
        log(f"[{leg}] errors {L['errors']}")

        if not args.no_extras:
            def timed(fn, reps=reps):
                fn()
                torch.cuda.synchronize()
                a0, z0 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a0.record()
                for _ in range(reps):
                    fn()
                z0.record()
                torch.cuda.synchronize()
                return a0.elapsed_time(z0) / reps

            def copy_in():
                At[:n, :n].copy_(A)

            def enc():
                copy_in()
                q.encode(At)

            # the factorization overwrites A~, so each timed factorization
            # starts from a fresh copy of A and its encoding; T_enc is the
            # encoding alone (the input copy timed on its own and subtracted)
            t_copy = timed(copy_in)
            t_enc_in = timed(enc)
            t_enc = t_enc_in - t_copy
            t_fac = timed(lambda: (enc(), q.factor(At, R))) - t_enc_in
            t_post = timed(lambda: q.postorth(At, Qpost, B, Bpost))
            L["overhead"] = {"T_enc_ms": round(t_enc, 4), "T_factor_coded_ms": round(t_fac, 4),
                             "T_post_ms": round(t_post, 4), "T_input_copy_ms": round(t_copy, 4)}
            if li == 0:
                # coded solve R_1 x = (G_0 Q_1)^T (G_0 b) on the last step's factors
                X = cqr.col_major(n, 1, dev)
                ws_solve = q.solve_workspace(1)
                step()
                t_solve = timed(lambda: q.solve(Qpost, R, Bpost, X, ws_solve))
                x_direct = torch.linalg.solve(A, B)
                out["solve"] = {"ms": round(t_solve, 4), "rel_err_vs_direct":
                                (torch.linalg.norm(X - x_direct) / torch.linalg.norm(x_direct)).item()}
                del X, ws_solve, x_direct
            log(f"[{leg}] coded legs done")

            # profiled pass: per-kernel HIP events on the library's streams
            q.profile(True)
            step()
            torch.cuda.synchronize()
            rep = q.profile_report()
            q.profile(False)
            phases = {k2: {"ms": round(r["ms"], 4), "launches": r["launches"],
                           "avg_us": round(1e3 * r["ms"] / max(r["launches"], 1), 3),
                           "tflops": round(r["flops"] / max(r["ms"], 1e-9) / 1e9, 3),
                           "gbs": round(r["bytes"] / max(r["ms"], 1e-9) / 1e6, 1)}
                      for k2, r in rep.items() if r["launches"]}
            L["phases"] = phases
            L["overhead"]["T_recov_ms_per_event"] = round(rep["recover"]["ms"] / max(len(sched), 1), 4)
            if li == 0:
                out["roofline"] = roofline_of(rep, b, leg, args.workload)
        q.close()

        if not args.no_extras and not args.skip_uncoded:
            # uncoded: same library and precision, K = 0, with the coded plan
            # released first (each plan's lookahead holds two streams; with both
            # plans alive there are more streams than the device's four hardware
            # queues, and the uncoded plan's streams could serialize)
            cu = cqr.Config(n, n, pr, pr, 0, 0, b, storage, reproject=reproject, lookahead=args.lookahead,
                            precision=PRECISIONS[leg]["code"], panel=panel)
            qu = cqr.CodedQR(cu, None, None, dev)
            Au, Ru = qu.alloc()

            def fac_u():
                Au.copy_(A)
                qu.factor(Au, Ru)
            t_copy_u = timed(lambda: Au.copy_(A))
            t_fu = timed(fac_u) - t_copy_u
            ov = L["overhead"]
            ov.update({"T_factor_uncoded_ms": round(t_fu, 4),
                       "overhead_pct": round(100 * (ov["T_enc_ms"] + ov["T_factor_coded_ms"] + ov["T_post_ms"] - t_fu)
                                             / t_fu, 2),
                       "floor_pct": round(100 * floor, 2),
                       "uncoded_tflops": round(F_unc / (t_fu * 1e-3) / 1e12, 4)})
            qu.close()
            del Au, Ru
            torch.cuda.empty_cache()
            log(f"[{leg}] uncoded leg done")
        out["legs"][leg] = L

    L0 = out["legs"][legs[0]]
    out["value"] = L0["tflops"]
    out["ms_per_step"] = L0["ms_per_step"]
    out["errors"] = L0["errors"]
    if "overhead" in L0:
        out["overhead"] = L0["overhead"]
    if len(legs) > 1:
        out["mixed_vs_fp64"] = {
            leg: {"speedup": round(L0["ms_per_step"] / out["legs"][leg]["ms_per_step"], 4),
                  "orth_coded": out["legs"][leg]["errors"]["orth_coded"],
                  "residual": out["legs"][leg]["errors"]["residual"]}
            for leg in legs[1:]}
    del first, At, R, Qpost, Bpost, A, B
    torch.cuda.empty_cache()

    if args.calib_copy:
        # reference for rocprofv3 FETCH_SIZE / WRITE_SIZE: reads and writes exactly 512 MiB each
        xs = torch.ones(64 << 20, dtype=torch.float64, device=dev)
        ys = torch.empty_like(xs)
        torch.cuda.synchronize()
        torch.mul(xs, 2.0, out=ys)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = 8 * (64 << 20)
        del xs, ys

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, w, F)
        log("cpu baseline done")
    print(json.dumps(out), flush=True)


PRECISIONS = {
    "fp64": {"code": 0, "dtype": "f64", "desc": "FP64 throughout"},
    "fp32": {"code": 1, "dtype": "f64 (R_bar on FP32 MFMA)",
             "desc": "coefficient product R_bar = Qbar^T Q_t on FP32 MFMA (FP32 sums over 16 k-values, FP64 "
                     "across them); rank-b update, re-projection, panels, decode, post-orth in FP64"},
    "bf16x3": {"code": 2, "dtype": "f64 (R_bar as split-BF16 products on BF16 MFMA)",
               "desc": "coefficient product R_bar = Qbar^T Q_t with each FP64 operand split into three BF16 parts, "
                       "six part products on BF16 MFMA (FP32 sums over 32 k-values, FP64 across them); rank-b "
                       "update, re-projection, panels, decode, post-orth in FP64"},
}


def kernel_of(phase: str, b: int, leg: str) -> str:
    """Kernel symbol behind a single-kernel phase (kernels are template-tagged per use)."""
    k = KERNEL_OF[phase]
    if phase == "trailing_update" and b >= 128:
        # K = b >= 128 and every trailing update spans the checksum columns
        # (>= 256 of them): the 128 x 128-tile form
        k = "nnq_kernel<0>"
    if phase == "trailing_product" and b > 64:
        # panels of several tile rows: 128 x 128 per workgroup, in FP64, in
        # FP32 (FP32 slabs in LDS) or as split-BF16 products
        k = {"fp64": "tnq_kernel<0>", "fp32": "tnf_kernel", "bf16x3": "tnb_kernel<0>"}[leg]
    elif phase == "trailing_product" and leg in ("fp32", "bf16x3"):
        # one tile row: the FP32 form of the LDS-staged product (the split-BF16
        # mode takes it too for such products)
        k = k.replace("<0, false>", "<0, true>")
    return k


def roofline_of(rep: dict, b: int, leg: str, workload: str) -> dict:
    """Roofline of the kernel holding the most time among phases that are exactly
    one kernel symbol (so rocprofv3's per-kernel average describes the same
    launches): algorithmic flops (or bytes) of its launches / their summed
    HIP-event durations on the stream they ran on."""
    dom = max((k for k in SINGLE_KERNEL_PHASES if rep[k]["launches"]), key=lambda k: rep[k]["ms"])
    r = rep[dom]
    f32_product = leg == "fp32" and dom == "trailing_product"
    mfma_peak = PEAK["fp32_mfma_tflops" if f32_product else "fp64_mfma_tflops"]
    # the rank-b update moves 16 bytes (read and write of C) per 2b flops:
    # MFMA-bound when b/8 flop/B exceeds the ridge peak / HBM bandwidth
    update_mfma = dom == "trailing_update" and b / 8.0 > mfma_peak * 1e3 / PEAK["hbm_gbs"]
    if dom in MFMA_PHASES or update_mfma:
        ach = r["flops"] / (r["ms"] * 1e-3) / 1e12
        roof = {"kernel": kernel_of(dom, b, leg), "phase": dom, "bound": "mfma", "achieved": round(ach, 3),
                "peak": mfma_peak, "unit": "TFLOP/s", "frac": round(ach / mfma_peak, 4)}
    else:
        ach = r["bytes"] / (r["ms"] * 1e-3) / 1e9
        roof = {"kernel": kernel_of(dom, b, leg), "phase": dom, "bound": "hbm", "achieved": round(ach, 1),
                "peak": PEAK["hbm_gbs"], "unit": "GB/s", "frac": round(ach / PEAK["hbm_gbs"], 4)}
    roof["avg_launch_us"] = round(1e3 * r["ms"] / r["launches"], 3)
    roof["launches"] = r["launches"]
    roof["flops_per_launch"] = r["flops"] / r["launches"]
    roof["share_of_profiled_step"] = round(r["ms"] / sum(x["ms"] for x in rep.values()), 3)
    roof["traffic"] = traffic_record(dom, workload) if leg == "fp64" else None
    roof["events_per_step"] = 2 * sum(x["launches"] for x in rep.values())
    return roof


def cpu_baseline(args, w: dict, F_workload: float) -> dict:
    """The FP64 oracle (plain numpy, unchanged) on the host cores, on a bounded
    sample: the full oracle step (encode, ICGS factor with the workload's kind
    of failures, recovery, post-orth) of the same workload, or, for workloads
    the host cannot finish in about half a minute, of the same grid, code and
    failure pattern at a reduced n (same block count and panel width, smaller
    blocks).  Its rate in the metric's unit is model flops / time."""
    import contextlib
    import platform
    import subprocess
    from oracle import coded_qr as oc
    n, pr, K, b = w["n"], w["pr"], w["K"], w["b"]
    n_s = n if n <= 4096 else max(16 * pr, min(n, w.get("cpu_sample_n", 4096)))
    inp = workload_inputs_at(w, n_s, args.seed)
    lay = oc.Layout(n_s, n_s, pr, pr, K, K, w["storage"])
    prob = oc.Problem(inp["A"], lay, inp["v"], inp["gh"], oc.FactorOptions(b, "icgs"), inp["schedule"], inp["rhs"])
    F_s = model_flops(lay.mp, n_s, lay.N - n_s, b)
    limit = contextlib.nullcontext()
    blas = {}
    cores = os.cpu_count()
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        info = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if info:
            cores = max(i.get("num_threads", 1) for i in info)
            blas = {"library": info[0].get("internal_api"), "version": info[0].get("version"),
                    "threading": info[0].get("threading_layer")}
        if args.cpu_threads > 0:
            limit = threadpool_limits(limits=args.cpu_threads)
            cores = args.cpu_threads
    except Exception:
        pass
    model = platform.processor() or ""
    try:
        for line in subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout.splitlines():
            if line.startswith("Model name"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    reps = 1 if n_s >= 4096 else max(1, int(10.0 / max(1e-3, 1e-11 * F_s)))
    with limit:
        t0 = time.perf_counter()
        for _ in range(reps):
            oc.run(prob)
        tc = (time.perf_counter() - t0) / reps
    rate = F_s / tc / 1e12
    sample = (f"{reps} full oracle step(s) (encode, ICGS factor with the workload's failure pattern, recovery, "
              f"post-orth) at n={n_s} on the workload's {pr}x{pr} grid, b={b}, K={K} {w['storage']}-node, "
              f"{tc:.2f} s each")
    res = {"value": round(rate, 5), "unit": "TFLOP/s", "cores": cores, "kind": "oracle", "sample": sample,
           "cpu_model": model, "blas": blas, "host_cpus": os.cpu_count()}
    if n_s != n:
        res["extrapolated_step_s"] = round(F_workload / (rate * 1e12), 1)
        res["extrapolation"] = "the workload's step time at this rate (model flops / rate); labelled extrapolated"
    return res


def workload_inputs_at(w: dict, n: int, seed: int) -> dict:
    """workload_inputs for the workload's grid, code and failure pattern at
    another n (the oracle's bounded CPU sample)."""
    pr, K, b = w["pr"], w["K"], w["b"]
    # the failure tolerance of the workload's code (in-node: the largest f with
    # f + f ceil(f / (p_r - f)) <= K)
    ftol = K if w["storage"] == "out" else max(
        f for f in range(1, pr) if f + f * (-(-f // (pr - f))) <= K)
    return {
        "A": synth.gaussian(n, n, seed),
        "rhs": synth.gaussian(n, 1, seed + 1),
        "v": synth.q_generator_draws(K, pr, seed),
        "gh": synth.r_generator_draws(pr, K, seed),
        "schedule": synth.draw_schedule(w["kind"], n // b, pr, pr, seed, nfail=w["nfail"], every=16, f=ftol),
    }


if __name__ == "__main__":
    main()
