"""Benchmark: prescribed-index reflectors per second on one MI355X.

Workload: the 2-D periodic Allen-Cahn Hessian on a 64 x 64 grid (d = 4096,
eps = 0.05, seeded field, seed 0), target index k = 5, midpoint shift
supplied (the shift the policy of section 4.3 hands to the sign kernels,
taken from the oracle's eigenvalues stored in tests/golden).  One step = one
reflector R_k from H resident in HBM to R resident in HBM.

  value        reflectors/s of the mixed path (split-BF16 MFMA bulk + FP64
               correction), which must reach ||R - R_k||_F <= 1e-8 sqrt(d)
  fp64_nsd     the plain FP64 Newton-Schulz iteration on the same input, run
               to the same accuracy (||X^2 - I||_F <= 1e-8 sqrt(d))
  with_shift_estimate  the same mixed solve with the shift estimated on the
               GPU by block Lanczos (setup included: the right-hand
               convention of the paper's timing comparison)
  roofline     the dominant kernel (the bulk BF16-word product), from HIP
               events around every launch in the timed region
  cpu_baseline the oracle (FP64 cyclic Jacobi) on the host cores: one sweep
               of the same matrix, scaled by the sweep count of a full solve,
               with a measured anchor (a full solve at d = 1024)

    python bench.py [--gpus 1] [--steps 5] [--warmup 2]

With --workload grad it times the gradient of L = <G, R_m(H)> (forward FP64
iteration to ||X^2 - I||_F < 1e-10 plus the checkpointed reverse sweep) on a
planted d = 2048, k = 10, gap 0.05 Hessian with G symmetric N(0, 1), and
prints its own JSON line.

With --workload batched it times the batched solve instead: 256 planted
problems (d uniform over 128/256/512/1024, k uniform in 1..16, relative gap
log-uniform in [1e-3, 1e-1], midpoint shifts, seed 0) in FP32 with the FP64
certificate, one refl_sign_batched call per step, against the same problems
solved one refl_sign call at a time; it prints its own JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "reflectors/s + MFMA TFLOP/s at d=4096, mixed vs FP64 NS, ‖R−R_k‖_F≤1e-8√d"
BF16_PEAK = 2.5e15
FP64_PEAK = 78.6e12


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def emit(out, args):
    """Print the JSON line; with --log also append it, stamped with the UTC
    time and host name, to that JSONL file (one row per run)."""
    print(json.dumps(out), flush=True)
    if getattr(args, "log", None):
        import platform
        row = dict(out, time_utc=time.strftime("%Y-%m-%dT%H:%M:%SZ", time.gmtime()),
                   host=platform.node())
        with open(args.log, "a") as f:
            f.write(json.dumps(row) + "\n")


def measured_traffic():
    """HBM bytes per launch of the bulk products from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE passes scaled by the copy-kernel
    calibration), or None when the product source changed since the counters
    were taken (the summary records the hash of the source it measured)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "gemm_words_pmc_allen_cahn_d4096.md")
    src = [os.path.join(ROOT, "paper_2605_24840_amd", "csrc", f) for f in ("gemm_w.hip", "common.h")]
    try:
        fields = {}
        for line in open(path):
            if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "source_sha256"):
                k, v = line.split(":", 1)
                fields[k] = v.strip()
        sha = hashlib.sha256(b"".join(open(f, "rb").read() for f in src)).hexdigest()
    except OSError:
        return None
    if fields.get("source_sha256") != sha or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--k", type=int, default=5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--words", type=int, default=2)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--lanczos-steps", type=int, default=3, help="timed solves with the shift estimated")
    ap.add_argument("--cg-tol", type=float, default=None, help="inner solve tolerance (library default if unset)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", choices=("allen_cahn", "batched", "grad", "kscan"), default="allen_cahn")
    ap.add_argument("--batch", type=int, default=256, help="problems of the batched workload")
    ap.add_argument("--profile", action="store_true",
                    help="counter-collection workload: one mixed solve, then a 256 MiB elementwise "
                         "kernel (reads 256 MiB, writes 256 MiB) that calibrates FETCH_SIZE/WRITE_SIZE")
    ap.add_argument("--log", default=os.environ.get("REFL_BENCH_LOG"),
                    help="also append the JSON line, with the time and host, to this JSONL file "
                         "(default: $REFL_BENCH_LOG, none if unset)")
    args = ap.parse_args()
    if args.steps < 1 or args.fp64_steps < 1 or args.lanczos_steps < 1:
        ap.error("--steps, --fp64-steps and --lanczos-steps must be at least 1")
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the reflector of one Hessian "
              "is computed on a single device; see the design notes for how it would shard.",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload == "grad":
        bench_grad(args)
        return
    if args.workload == "kscan":
        bench_kscan(args)
        return

    import torch
    from paper_2605_24840_amd import inputs, refl

    k, seed = args.k, args.seed
    golden = np.load(os.path.join(ROOT, "tests", "golden", f"allen_cahn_n64_seed{seed}.npz"))
    H, u = inputs.allen_cahn_2d(64, float(golden["eps"]), seed)
    assert np.array_equal(u, golden["u"]), "input generator does not reproduce the stored field"
    d = H.shape[0]
    w, Vk = golden["w"], golden["V"][:, :k]
    s = 0.5 * (w[k - 1] + w[k])
    target = 1e-8 * np.sqrt(d)
    log(f"workload d={d} k={k} s={s:.6f} gap={w[k] - w[k - 1]:.4e} target={target:.2e}")

    dev = torch.device("cuda", 0)
    Hg = torch.from_numpy(H).to(dev)
    R = torch.empty((d, d), dtype=torch.float64, device=dev)
    h = refl.Handle(dev)
    # The product launches are timed by HIP events in the timed solves, on
    # every fourth bulk step (a sample of about a quarter of the launches):
    # an event pair around every product cost about 0.25 ms per solve.
    mixed_kw = dict(precision="mixed", words=args.words, tol=target, timing=4)
    if args.cg_tol is not None:
        mixed_kw["cg_tol"] = args.cg_tol
    fp64_kw = dict(precision="fp64", tol=target, timing=True)
    h.reserve(d, refl.make_params(k, s, **mixed_kw))

    def run(kw):
        _, info, st = refl.sign(Hg, k, s, handle=h, out=R, check=False, **kw)
        if st != 0:
            raise RuntimeError(f"refl_sign returned {refl.STATUS[st]}: {refl.refl_last_error(h.h)}")
        return info

    def err_vs_oracle():
        Rn = R.cpu().numpy()
        Rn -= np.eye(d)
        Rn += 2.0 * Vk @ Vk.T
        return float(np.linalg.norm(Rn))

    if args.profile:
        info = run(mixed_kw)
        log(f"profile solve: {info['ms_total']:.2f} ms, steps={info['ns_steps']}")
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        log("calibration kernel done (256 MiB read + 256 MiB write per launch)")
        h.close()
        return

    # ---- mixed path ----
    for i in range(args.warmup):
        info = run(mixed_kw)
        log(f"warmup {i}: {info['ms_total']:.2f} ms")
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        infos.append(run(mixed_kw))
    torch.cuda.synchronize()
    t_mixed = (time.perf_counter() - t0) / args.steps
    err_mixed = err_vs_oracle()
    last = infos[-1]
    log(f"mixed: {1e3 * t_mixed:.2f} ms/reflector, steps={last['ns_steps']} sweeps={last['polish_sweeps']} "
        f"cg={last['cg_iters']} dk={last['dk_bound']:.1e} bulk={last['ms_bulk']:.2f} polish={last['ms_polish']:.2f} err={err_mixed:.2e}")
    nprod = {1: 1, 2: 3, 3: 6}[args.words]
    gemm_ms = sum(i["ms_gemm"] for i in infos)
    gemm_n = sum(i["gemm_launches"] for i in infos)
    avg_launch_s = gemm_ms / gemm_n / 1e3
    # Algorithmic work of one symmetric product (d^2/2 outputs x 2d flop):
    # d^3, whatever arithmetic carries it.  The split-word product executes
    # it once per kept word product (nprod d^3), and the matrix cores issue
    # that over the padded upper tiles (full diagonal tiles, K rounded to 32).
    flop_launch = float(d) ** 3
    achieved = flop_launch / avg_launch_s
    word_flop_launch = nprod * flop_launch
    ts = int(last["bulk_tile"])
    nt = -(-d // ts)
    issued_flop_launch = nprod * (nt * (nt + 1) // 2) * ts * ts * 2.0 * (-(-d // 32) * 32)
    steps_mixed = float(np.mean([i["ns_steps"] for i in infos]))
    bulk_alg_tflops = steps_mixed * 2 * float(d) ** 3 / (np.mean([i["ms_bulk"] for i in infos]) / 1e3) / 1e12

    # ---- mixed path with the shift estimated by block Lanczos ----
    lz_kw = dict(mixed_kw)
    h.reserve(d, refl.make_params(k, None, **lz_kw))

    def run_lz():
        _, info, st = refl.sign(Hg, k, None, handle=h, out=R, check=False, seed=seed, **lz_kw)
        if st != 0:
            raise RuntimeError(f"refl_sign (Lanczos shift) returned {refl.STATUS[st]}: {refl.refl_last_error(h.h)}")
        return info

    run_lz()
    torch.cuda.synchronize()
    tl = time.perf_counter()
    infos_lz = [run_lz() for _ in range(args.lanczos_steps)]
    torch.cuda.synchronize()
    t_lz = (time.perf_counter() - tl) / args.lanczos_steps
    err_lz = err_vs_oracle()
    il = infos_lz[-1]
    log(f"mixed + Lanczos shift: {1e3 * t_lz:.2f} ms/reflector, lanczos steps={il['lanczos_steps']} "
        f"setup={il['ms_setup']:.2f} ms s={il['s']:.9f} eps={il['eps']:.2e} err={err_lz:.2e}")

    # ---- plain FP64 iteration to the same accuracy ----
    info64 = run(fp64_kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    infos64 = [run(fp64_kw) for _ in range(args.fp64_steps)]
    torch.cuda.synchronize()
    t_fp64 = (time.perf_counter() - t1) / args.fp64_steps
    err_fp64 = err_vs_oracle()
    g64 = sum(i["ms_gemm"] for i in infos64) / sum(i["gemm_launches"] for i in infos64) / 1e3
    fp64_achieved = float(d) ** 3 / g64
    log(f"fp64: {1e3 * t_fp64:.2f} ms/reflector, steps={infos64[-1]['ns_steps']} err={err_fp64:.2e} "
        f"gemm {1e3 * g64:.3f} ms/launch = {fp64_achieved / 1e12:.1f} TFLOP/s")
    del info64

    # ---- oracle on the host cores ----
    cpu = None
    if not args.no_cpu:
        cpu = cpu_oracle(H, int(golden["sweeps"]))

    out = {
        "metric": METRIC,
        "value": 1.0 / t_mixed,
        "unit": "reflectors/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_mixed,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"bf16x{nprod} (f32 accumulate) + f64 correction",
        "data": "synthetic",
        "config": {"workload": "allen_cahn_2d_periodic", "n": 64, "d": d, "eps": float(golden["eps"]),
                   "seed": seed, "k": k, "shift": "supplied midpoint", "scale": "inf-norm",
                   "words": args.words},
        "err_fro": err_mixed,
        "err_target": target,
        "ns_steps": last["ns_steps"],
        "polish_sweeps": last["polish_sweeps"],
        "cg_iters": last["cg_iters"],
        "dk_bound": last["dk_bound"],
        "ms_bulk": float(np.mean([i["ms_bulk"] for i in infos])),
        "ms_polish": float(np.mean([i["ms_polish"] for i in infos])),
        "bulk_algorithmic_tflops": bulk_alg_tflops,
        "fp64_ns": {"value": 1.0 / t_fp64, "unit": "reflectors/s", "ms_per_step": 1e3 * t_fp64,
                    "ns_steps": infos64[-1]["ns_steps"], "err_fro": err_fp64,
                    "gemm_tflops": fp64_achieved / 1e12, "gemm_frac_of_fp64_peak": fp64_achieved / FP64_PEAK},
        "speedup_vs_fp64": t_fp64 / t_mixed,
        "with_shift_estimate": {"value": 1.0 / t_lz, "unit": "reflectors/s", "ms_per_step": 1e3 * t_lz,
                                "lanczos_steps": il["lanczos_steps"], "ms_setup": il["ms_setup"],
                                "s": il["s"], "eps": il["eps"], "margin": il["margin"], "err_fro": err_lz},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": BF16_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / BF16_PEAK, "traffic": measured_traffic(),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, calibrated)",
                     "kernel": f"k_sym_gemm_wd<{args.words}, GEMM_RESIDUAL|GEMM_UPDATE, {ts}>",
                     "launches": gemm_n, "avg_launch_ms": 1e3 * avg_launch_s,
                     "flop_per_launch": flop_launch,
                     "flop_per_launch_meaning": "algorithmic: d^3 per symmetric product",
                     "word_product_flop_per_launch": word_flop_launch,
                     "word_product_tflops": word_flop_launch / avg_launch_s / 1e12,
                     "word_product_frac": word_flop_launch / avg_launch_s / BF16_PEAK,
                     "mfma_issued_flop_per_launch": issued_flop_launch,
                     "mfma_issued_frac": issued_flop_launch / avg_launch_s / BF16_PEAK},
        "cpu_baseline": cpu,
    }
    h.close()
    emit(out, args)


FP32_PEAK = 157.3e12


def cpu_oracle(H, sweeps_full):
    """The oracle (FP64 cyclic Jacobi, then R_k from its eigenvectors) on the
    host cores.  The d = 4096 figure is one sweep of this matrix times the
    sweep count of its full solve (stored with the golden eigenvectors).
    Anchor at d = 1024 (planted, gap 0.02): a full solve and one sweep with
    all threads, so that full-solve time / (sweeps x first sweep) checks
    the extrapolation, and one sweep on one thread."""
    import oracle
    from paper_2605_24840_amd import inputs
    d = H.shape[0]
    nthr = oracle.oracle_threads()
    tc = time.perf_counter()
    oracle.jacobi_eigh(H, max_sweeps=1)
    t_sweep = time.perf_counter() - tc
    log(f"cpu oracle: {t_sweep:.1f} s/sweep at d={d} on {nthr} threads")
    Ha, lam, Q = inputs.planted_hessian(1024, 8, 0.02, 0)
    tc = time.perf_counter()
    w, V, sw_a = oracle.jacobi_eigh(Ha)
    oracle.reflector_from_eig(V, 8)
    t_full_a = time.perf_counter() - tc
    tc = time.perf_counter()
    oracle.jacobi_eigh(Ha, max_sweeps=1)
    t_sweep_a = time.perf_counter() - tc
    oracle.set_oracle_threads(1)
    tc = time.perf_counter()
    oracle.jacobi_eigh(Ha, max_sweeps=1)
    t_sweep_a1 = time.perf_counter() - tc
    oracle.set_oracle_threads(nthr)
    log(f"cpu oracle d=1024: full solve {t_full_a:.2f} s ({sw_a} sweeps), one sweep {t_sweep_a:.2f} s on "
        f"{nthr} threads, {t_sweep_a1:.2f} s on one thread")
    return {"value": 1.0 / (t_sweep * sweeps_full), "unit": "reflectors/s", "cores": nthr, "kind": "oracle",
            "sample": f"one cyclic-Jacobi sweep of this d={d} matrix ({t_sweep:.1f} s on {nthr} threads) "
                      f"scaled by the {sweeps_full} sweeps of its full solve",
            "anchor_d1024": {"full_solve_s": t_full_a, "sweeps": sw_a, "one_sweep_s": t_sweep_a,
                             "full_over_sweeps_times_first": t_full_a / (sw_a * t_sweep_a),
                             "one_sweep_single_thread_s": t_sweep_a1, "threads": nthr,
                             "reflectors_per_s": 1.0 / t_full_a}}


def bench_grad(args):
    """Gradients/s of refl_sign_grad on the differentiation workload, the
    derivative products against the FP64 MFMA peak, and the oracle's reverse
    sweep on the host cores."""
    import torch
    from paper_2605_24840_amd import inputs, refl

    d, k, gap, seed = 2048, 10, 0.05, args.seed
    H, lam, Q = inputs.planted_hessian(d, k, gap, seed)
    G = inputs.symmetric_normal(d, seed)
    s = 0.5 * (lam[k - 1] + lam[k])
    dev = torch.device("cuda", 0)
    Hg, Gg = torch.from_numpy(H).to(dev), torch.from_numpy(G).to(dev)
    h = refl.Handle(dev)
    kw = dict(precision="fp64", tol=1e-10, timing=True)

    def run():
        g, loss, _, info, st = refl.sign_grad(Hg, Gg, k, s, handle=h, check=False, **kw)
        if st != 0:
            raise RuntimeError(f"refl_sign_grad returned {refl.STATUS[st]}: {refl.refl_last_error(h.h)}")
        return g, loss, info

    for i in range(args.warmup):
        _, _, info = run()
        log(f"warmup {i}: {info['ms_total']:.2f} ms")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [run() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.steps
    g, loss, info = runs[-1]
    m, alpha = info["ns_steps"], info["alpha"]
    deriv_flop = 5.0 * float(d) ** 3 * m      # per gradient: m steps of -X Gb (2 d^3) + three-pair (3 d^3)
    gemm_s = np.mean([r[2]["ms_gemm"] for r in runs]) / 1e3
    achieved = deriv_flop / gemm_s
    # Directional derivative against central differences (alpha, m fixed).
    E = inputs.symmetric_normal(d, seed + 1)
    E /= np.linalg.norm(E)
    Eg = torch.from_numpy(E).to(dev)
    tstep = 1e-4

    def L(Hx):
        Rx, _, st = refl.sign(Hx, k, s, handle=h, alpha=alpha, fixed_steps=m)
        return float((Gg * Rx).sum())
    fd = (L(Hg + tstep * Eg) - L(Hg - tstep * Eg)) / (2 * tstep)
    dd = float((g * Eg).sum())
    fd_rel = abs(dd - fd) / abs(fd)
    log(f"grad: {1e3 * t_step:.2f} ms per gradient, m={m}, forward {info['ms_bulk']:.2f} ms, "
        f"derivative {info['ms_polish']:.2f} ms; derivative products {1e3 * gemm_s:.2f} ms = "
        f"{achieved / 1e12:.1f} TFLOP/s; central-difference check {fd_rel:.2e}")

    # The gradient of the limit through a MIXED forward (split-BF16 bulk,
    # FP64 correction, projected FP64 solves on the certified eigenspace).
    kwm = dict(precision="mixed", tol=1e-8 * np.sqrt(d))

    def run_mixed():
        gm, lm, _, infm, stm = refl.sign_grad(Hg, Gg, k, s, handle=h, check=False, **kwm)
        if stm != 0:
            raise RuntimeError(f"refl_sign_grad (mixed) returned {refl.STATUS[stm]}: {refl.refl_last_error(h.h)}")
        return gm, infm

    for _ in range(max(1, args.warmup)):
        run_mixed()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs_m = [run_mixed() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_mixed = (time.perf_counter() - t0) / args.steps
    gm, infm = runs_m[-1]
    dd_m = float((gm * Eg).sum())
    mixed = {"value": 1.0 / t_mixed, "unit": "gradients/s", "ms_per_step": 1e3 * t_mixed,
             "what": "gradient of the limit <G, R_k(H)> (MIXED forward, projected FP64 solves)",
             "ns_steps": infm["ns_steps"], "bulk_words": infm["bulk_words"], "cg_iters": infm["cg_iters"],
             "directional_vs_fp64_chain_rel": abs(dd_m - dd) / abs(dd),
             "rel_diff_vs_fp64_chain": float(torch.linalg.norm(gm - g) / torch.linalg.norm(g))}
    log(f"grad mixed: {1e3 * t_mixed:.2f} ms per gradient, steps={infm['ns_steps']} cg={infm['cg_iters']}, "
        f"relative difference to the FP64 chain gradient {mixed['rel_diff_vs_fp64_chain']:.2e}")

    cpu = None
    if not args.no_cpu:
        import oracle
        X0 = (H - s * np.eye(d)) / alpha
        tc = time.perf_counter()
        X1 = oracle.ns_iterate(X0)
        t_fwd = time.perf_counter() - tc
        tc = time.perf_counter()
        oracle.ns_step_derivative(X1, G)
        t_rev = time.perf_counter() - tc
        t_cpu = m * (t_fwd + t_rev)
        cpu = {"value": 1.0 / t_cpu, "unit": "gradients/s", "cores": oracle.oracle_threads(),
               "kind": "oracle",
               "sample": f"one forward step ({t_fwd:.2f} s) and one reverse step ({t_rev:.2f} s) of the "
                         f"oracle's FP64 recurrences at d={d}, scaled by the {m} steps"}
        log(f"cpu oracle: {t_fwd:.2f} s forward step, {t_rev:.2f} s reverse step")
    h.close()
    out = {
        "metric": "gradients/s of <G, R_m(H)>, d=2048 (FP64 forward + reverse sweep)",
        "value": 1.0 / t_step,
        "unit": "gradients/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "planted_gradient", "d": d, "k": k, "gap": gap, "seed": seed,
                   "G": "symmetric N(0,1)", "tol": kw["tol"], "ckpt_every": 0, "iterates": "all kept (they fit in 16 GiB)"},
        "ns_steps": m,
        "ms_forward": info["ms_bulk"],
        "ms_derivative": info["ms_polish"],
        "central_difference_rel": fd_rel,
        "mixed_limit_gradient": mixed,
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": FP64_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK, "traffic": None,
                     "kernel": "k_sym_gemm_f<double, GEMM_PLAIN_NEG> + k_adjoint_step<double>",
                     "launches": info["gemm_launches"], "avg_launch_ms": 1e3 * gemm_s / max(info["gemm_launches"], 1)},
        "cpu_baseline": cpu,
    }
    emit(out, args)


def bench_kscan(args):
    """The target-index scan of section 5.3 at the paper's breadth: rotated
    quartic, d = 64, k in {1, 2, 4, 8, 16}, 32 matched starts, converged
    engine and midpoint filters m = 2, 4, 6 (outer.target_index_scan); the
    success rate, the median wall time per outer step and per run, and the
    median one-step direction error over 32 local perturbations.  The value is
    outer steps per second over the whole scan."""
    import torch
    from paper_2605_24840_amd import outer, refl

    dev = torch.device("cuda", 0)
    h = refl.Handle(dev)
    outer.target_index_scan(h, ks=(1,), nstarts=1, ms=(2,), npert=1)     # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = outer.target_index_scan(h, nstarts=32, npert=32)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    h.close()
    table, total_steps = {}, 0
    for k, per_k in res.items():
        row = {}
        for m, r in per_k.items():
            total_steps += sum(r["steps"])
            name = "exact" if m == 0 else f"m{m}"
            row[name] = {"success_rate": sum(r["success"]) / len(r["success"]),
                         "median_ms_per_step": r["ms_per_step"],
                         "median_ms_per_run": float(np.median(r["ms_per_run"])),
                         "median_direction_error": float(np.median(r["dir_err"]))}
            log(f"k={k:2d} {name:5s}: success {sum(r['success'])}/{len(r['success'])}, "
                f"{r['ms_per_step']:.3f} ms/step, direction error {np.median(r['dir_err']):.2e}")
        table[str(k)] = row
    out = {
        "metric": "outer steps/s of the section 5.3 target-index scan (d=64, 32 starts, exact + p_2, p_4, p_6)",
        "value": total_steps / t_all,
        "unit": "outer steps/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": 1e3 * t_all,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "rotated_quartic_scan", "d": 64, "ks": [1, 2, 4, 8, 16], "starts": 32,
                   "eta": 0.3, "max_steps": 200, "perturbations": 32, "perturbation_scale": 0.05,
                   "shift": "exact midpoint (dense eigensolver)"},
        "scan": table,
        "roofline": None,
        "cpu_baseline": None,
    }
    emit(out, args)


def bench_batched(args):
    """Batched planted solves (FP32 bulk, FP64 certificate): problems/s of one
    refl_sign_batched call with the inputs resident in HBM, the same problems
    through refl_sign one at a time, and the grouped product kernels against
    the FP32 MFMA peak."""
    import torch
    from paper_2605_24840_amd import inputs, refl

    n, seed = args.batch, args.seed
    specs = inputs.batch_specs(n, seed=seed)
    dev = torch.device("cuda", 0)
    log(f"batched workload: {n} problems, generating")
    Hs, ks, ss, Qs = [], [], [], {}
    sample = {}
    for p, spec in enumerate(specs):
        H, lam, Q = inputs.batch_problem(spec)
        k = spec[1]
        Hs.append(torch.from_numpy(H).to(dev))
        ks.append(k)
        ss.append(0.5 * (lam[k - 1] + lam[k]))
        if spec[0] not in sample:
            sample[spec[0]] = (p, H, Q)
    ds = [spec[0] for spec in specs]
    Rs = [torch.empty_like(H) for H in Hs]
    h = refl.Handle(dev)
    kw = dict(precision="fp32", tol=1e-3)

    # Arguments marshalled once.  The timed calls run the steps as captured
    # HIP graphs; a second set of calls with per-launch timing events (which
    # runs the same steps eagerly) gives the grouped products' kernel time.
    call = refl.BatchedCall(Hs, ks, ss, Rs, **kw)
    call_t = refl.BatchedCall(Hs, ks, ss, Rs, timing=True, **kw)

    def run_batch(c):
        st = c.run(h.h, check=False)
        if st != 0:
            raise RuntimeError(f"refl_sign_batched returned {refl.STATUS[st]}: {refl.refl_last_error(h.h)}")
        return c.infos[0].ms_gemm   # no Python objects are built inside the timed loop

    for i in range(args.warmup):
        run_batch(call)
        log(f"warmup {i}: {call.infos[0].ms_total:.2f} ms")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run_batch(call)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.steps
    run_batch(call_t)
    gemm_ms = [run_batch(call_t) for _ in range(max(1, min(args.steps, 3)))]
    infos = [i.as_dict() for i in call_t.infos]
    steps = [i["ns_steps"] for i in infos]
    # Algorithmic work of the grouped FP32 products: a symmetric d x d
    # product is d^3 multiply-adds' worth of flops counted once (d^3 flops
    # for the upper half, as for the single-problem products); problem p
    # runs steps + 1 RESIDUAL and steps UPDATE products.  Orders up to
    # SMALL_MAX run in the LDS-resident launch, outside the grouped products
    # and their timing events.
    flop = sum((2 * st + 1) * float(d) ** 3 for st, d in zip(steps, ds) if d > refl.SMALL_MAX["fp32"])
    gemm_s = float(np.mean(gemm_ms)) / 1e3
    launches = infos[0]["gemm_launches"]
    achieved = flop / gemm_s
    errs = {}
    for d, (p, H, Q) in sorted(sample.items()):
        Rk = np.eye(d) - 2.0 * Q[:, :ks[p]] @ Q[:, :ks[p]].T
        errs[str(d)] = float(np.linalg.norm(Rs[p].cpu().numpy() - Rk))
    log(f"batched: {1e3 * t_batch:.2f} ms per batch ({n / t_batch:.1f} problems/s), steps "
        f"{min(steps)}..{max(steps)}, grouped products {1e3 * gemm_s:.2f} ms in {launches} launches "
        f"= {achieved / 1e12:.1f} TFLOP/s; errors {errs}")

    # The same problems one refl_sign call at a time.
    def run_seq():
        for p in range(n):
            _, info, st = refl.sign(Hs[p], ks[p], ss[p], handle=h, out=Rs[p], check=False, **kw)
            if st != 0:
                raise RuntimeError(f"refl_sign returned {refl.STATUS[st]} on problem {p}")

    run_seq()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    run_seq()
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t1
    log(f"sequential: {1e3 * t_seq:.2f} ms ({n / t_seq:.1f} problems/s)")

    cpu = None
    if not args.no_cpu:
        import oracle
        # One full oracle solve per size, weighted by how often the size occurs.
        t_size = {}
        for d, (p, H, Q) in sorted(sample.items()):
            tc = time.perf_counter()
            oracle.jacobi_eigh(H)
            t_size[d] = time.perf_counter() - tc
            log(f"cpu oracle d={d}: {t_size[d]:.2f} s")
        t_avg = sum(t_size[d] for d in ds) / n
        cpu = {"value": 1.0 / t_avg, "unit": "problems/s", "cores": oracle.oracle_threads(),
               "kind": "oracle",
               "sample": "one full cyclic-Jacobi solve per size (" +
                         ", ".join(f"d={d}: {t:.2f} s" for d, t in sorted(t_size.items())) +
                         f"), weighted by the size mix of the {n} problems"}
    h.close()
    out = {
        "metric": "problems/s, batched planted solves (FP32 bulk + FP64 certificate)",
        "value": n / t_batch,
        "unit": "problems/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_batch,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 certificate)",
        "data": "synthetic",
        "config": {"workload": "batched_planted", "problems": n, "sizes": [128, 256, 512, 1024],
                   "kmax": 16, "grel": [1e-3, 1e-1], "seed": seed, "tol": kw["tol"],
                   "shift": "supplied midpoint"},
        "ns_steps": {"min": min(steps), "max": max(steps), "mean": float(np.mean(steps))},
        "err_fro_by_size": errs,
        "sequential": {"value": n / t_seq, "unit": "problems/s", "ms": 1e3 * t_seq},
        "speedup_vs_sequential": t_seq / t_batch,
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": FP32_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / FP32_PEAK, "traffic": None,
                     "kernel": "k_sym_gemm_f_grouped<float, GEMM_RESIDUAL|GEMM_UPDATE>",
                     "launches": launches, "avg_launch_ms": 1e3 * gemm_s / max(launches, 1)},
        "cpu_baseline": cpu,
    }
    emit(out, args)


if __name__ == "__main__":
    main()
