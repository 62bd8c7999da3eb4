"""Benchmark: f + grad evaluations per second of the split-CTMRG HIP path.

One step = one complete evaluation of the hot path for one PEPS tensor:
ctm_init (PEPO, D4 projection, product-boundary environments of both networks),
ctm_iterate until the corner-spectrum change drops below tol (or max_iter),
ctm_free_energy and ctm_grad.  The PEPS tensor is resident in HBM before the
timed region starts (a float64 torch tensor on cuda:0, passed by pointer).

Prints one JSON line (rank 0, one GPU).  Besides the throughput it reports
  roofline     the kernel class with the largest share of device time in one
               profiled evaluation (HIP events on the library's stream around
               every launch), its algorithmic rate and the matching peak;
  cpu_baseline the FP64 NumPy oracle (the same split-CTMRG steps) timed on the
               host cores on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from synth_inputs import WORKLOADS, raw_peps, workload_peps  # noqa: E402

T_START = time.perf_counter()
SERVING_MAX_ITER = 60

PEAK_FP64_MFMA_TFLOPS = 78.6      # MI355X dense FP64 matrix peak
PEAK_FP64_VECTOR_TFLOPS = 78.6    # MI355X FP64 vector peak (256 CU x 2.4 GHz x 128 flop/clk)

# kernel classes timed by the library's profile mode: name, roofline bound, peak
KERNEL_CLASSES = {
    0: ("gemm_f64_kernel (v_mfma_f64_16x16x4)", "mfma", PEAK_FP64_MFMA_TFLOPS),
    1: ("jacobi_reg_kernel / jacobi_svd_kernel", "alu", PEAK_FP64_VECTOR_TFLOPS),
    2: ("cholqr_reg_kernel / cholqr_kernel", "alu", PEAK_FP64_VECTOR_TFLOPS),
    3: ("gemm_lp_kernel (FP32 / BF16 MFMA)", "mfma", 157.3),
    4: ("gemm_reduce_kernel (split-K)", "hbm", None),
}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "d5_chi100_traffic.json")
KERNELS_SRC = os.path.join(ROOT, "paper_2506_19339_amd", "csrc", "kernels.hip")
ENGINE_SRC = os.path.join(ROOT, "paper_2506_19339_amd", "csrc", "engine.hip")
TRAFFIC_KEY = {0: "gemm_f64_kernel", 1: "jacobi_reg_kernel", 2: "cholqr_reg_kernel"}


def measured_traffic(cls):
    """HBM bytes per launch of the kernel class from the FETCH_SIZE / WRITE_SIZE
    counter runs recorded in profiles/ (scaled by the copy calibration), or
    None when they were taken with other kernel or engine source than the
    current one (the engine decides which products are launched)."""
    import hashlib
    try:
        data = json.load(open(TRAFFIC_FILE))
        cur_k = hashlib.sha256(open(KERNELS_SRC, "rb").read()).hexdigest()
        cur_e = hashlib.sha256(open(ENGINE_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    if (data.get("kernels_hip_sha256") != cur_k or data.get("engine_hip_sha256") != cur_e
            or TRAFFIC_KEY.get(cls) not in data["kernels"]):
        return None
    return data["kernels"][TRAFFIC_KEY[cls]]["hbm_bytes_per_launch"]


def gpu_eval(ctm, torch, w, A, g, stream, profile=False, precision=0, refine=False, method="split"):
    c = ctm.SplitCTM(w["beta"], A, w["chi"], max_iter=w["max_iter"], tol=w["tol"],
                     stream=stream, profile=profile, precision=precision, refine=refine, method=method)
    done, delta, conv = c.iterate(0)
    f, lk3, lk2 = c.free_energy()
    c.grad(g)
    return c, dict(iters=done, delta=delta, converged=conv, f=f)


def factor_kernels():
    """The kernels of a move timed alone through the self-test library (the
    register Cholesky-QR factor and one-sided Jacobi on three 128-wide
    problems per launch, as in a projector stage; the FP64 GEMM at the most
    frequent product shapes of a D = 5, chi = 100 evaluation, with and
    without the split-K plan)."""
    import ctypes
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2506_19339_amd", "libctm_selftest.so")
    if not os.path.exists(path):
        raise SystemExit("libctm_selftest.so is not built")
    lib = ctypes.CDLL(path)
    us = ctypes.c_double(0.0)

    def timed(fn, *a):
        rc = fn(*a, ctypes.byref(us))
        if rc != 0:
            raise SystemExit("self-test timing call failed (%d)" % rc)
        return us.value

    f = lib.ctm_selftest_time_factor
    for which, name in ((0, "cholqr_reg_kernel"), (1, "jacobi_reg_kernel with V"), (2, "jacobi_reg_kernel without V")):
        sweeps = 5 if which else 0
        t = timed(f, which, 128, 3, sweeps, 50 if which == 0 else 10)
        row = {"kernel": name, "k": 128, "problems_per_launch": 3, "us_per_launch": round(t, 1)}
        if which:
            row.update(sweeps=sweeps, us_per_sweep=round(t / sweeps, 1))
        print(json.dumps(row), flush=True)
    g = lib.ctm_selftest_time_gemm
    for M, N, K in ((4000, 2500, 1000), (1000, 1000, 1000), (10000, 500, 1000), (20000, 500, 500),
                    (1000, 2500, 1000), (2500, 500, 1000), (50000, 200, 100), (10000, 100, 1000),
                    (1000, 100, 1000), (500, 100, 10000)):
        t1 = timed(g, M, N, K, 1, 20)
        t0 = timed(g, M, N, K, 0, 20)
        fl = 2.0 * M * N * K
        print(json.dumps({"kernel": "gemm_f64", "M": M, "N": N, "K": K,
                          "us_split_plan": round(t1, 1), "tflops_split_plan": round(fl / t1 / 1e6, 1),
                          "us_no_split": round(t0, 1), "tflops_no_split": round(fl / t0 / 1e6, 1)}), flush=True)


def method_sweep(ctm, torch, steps, moves=20, skip=5):
    """Split-CTMRG against the reduced method on the same kernels (the runtime
    comparison of Sec. IV A): time per move of both networks for D = 2..6 at
    chi = D^2 and at chi = 100, measured over `moves` moves after `skip`
    untimed ones (moves to convergence depend on the tensor; per-move cost
    does not), and f after those moves."""
    beta = 0.22
    for chi_rule in ("D^2", "100"):
        for D in (2, 3, 4, 5, 6):
            chi = D * D if chi_rule == "D^2" else 100
            A = torch.from_numpy(raw_peps(D, 0)).cuda()
            row = dict(D=D, chi=chi, beta=beta, moves_timed=moves)
            for method in ("split", "reduced"):
                best = None
                for _ in range(max(1, steps)):
                    c = ctm.SplitCTM(beta, A, chi, max_iter=skip + moves, tol=0.0, method=method)
                    c.iterate(skip)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    c.iterate(moves)
                    torch.cuda.synchronize()
                    dt = (time.perf_counter() - t0) / moves
                    best = dt if best is None else min(best, dt)
                    f = c.free_energy()[0]
                    _, nbytes = c.query()
                    c.close()
                row[method] = dict(ms_per_move=1e3 * best, f=f, device_bytes=int(nbytes))
            row["split_over_reduced_time"] = row["split"]["ms_per_move"] / row["reduced"]["ms_per_move"]
            print(json.dumps(row), flush=True)


def cpu_baseline(name, sample_iters):
    """Oracle (FP64 NumPy, same wiring) on a bounded sample: the first
    `sample_iters` iterations of both networks of the workload, then the
    per-evaluation time is extrapolated with the GPU's iteration count."""
    from oracle import model, split
    w = WORKLOADS[name]
    A = model.d4_symmetrize(workload_peps(name))
    t_net = []
    for O in (model.pepo_O(w["beta"]), model.identity_pepo()):
        env = split.init_env(A.shape[1], O.shape[2])
        env, _ = split.step(env, A, O, split.GROW_CHI)
        times = []
        for _ in range(sample_iters):
            t0 = time.perf_counter()
            env, _ = split.step(env, A, O, w["chi"])
            times.append(time.perf_counter() - t0)
        t_net.append(float(np.mean(times)))
    return t_net


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="d5_chi100")
    ap.add_argument("--cpu-sample-iters", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile-pass", action="store_true")
    ap.add_argument("--no-fp32-leg", action="store_true")
    ap.add_argument("--no-reduced-leg", action="store_true")
    ap.add_argument("--no-lbfgs-leg", action="store_true")
    ap.add_argument("--lbfgs-steps", type=int, default=5)
    ap.add_argument("--no-serving-leg", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=256,
                    help="requests of the serving trace replayed in real time (Poisson, 20/s)")
    ap.add_argument("--reduced-only", action="store_true",
                    help="only time the reduced method on the workload (for profiling it alone)")
    ap.add_argument("--method-sweep", action="store_true",
                    help="only compare split-CTMRG with the reduced method: time per move for "
                         "D = 2..6 at chi = D^2 and chi = 100 (one JSON line per case)")
    ap.add_argument("--factor-kernels", action="store_true",
                    help="only time the factorisation kernels and the FP64 GEMM alone at the "
                         "shapes of a D = 5, chi = 100 move (one JSON line per case)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy three times (the reference "
                         "kernel for scaling FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": src.numel() * 8, "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU: the library has no multi-GPU path "
              "(independent evaluations would shard one per GPU)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2506_19339_amd import ctm

    if args.method_sweep:
        method_sweep(ctm, torch, args.steps)
        return
    if args.factor_kernels:
        factor_kernels()
        return
    if args.reduced_only:
        w = WORKLOADS[args.workload]
        A = torch.from_numpy(workload_peps(args.workload)).cuda()
        g = torch.empty_like(A)
        for i in range(args.warmup):
            c, _ = gpu_eval(ctm, torch, w, A, g, None, method="reduced")
            c.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            c, info = gpu_eval(ctm, torch, w, A, g, None, method="reduced")
            c.close()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / max(args.steps, 1)
        print(json.dumps(dict(method="reduced", workload=args.workload, s_per_eval=dt, iters=info["iters"],
                              f=info["f"])), flush=True)
        return

    w = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    A = torch.from_numpy(workload_peps(args.workload)).to(dev)
    g = torch.empty_like(A)
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    torch.cuda.synchronize()

    for i in range(args.warmup):
        t1 = time.perf_counter()
        c, info = gpu_eval(ctm, torch, w, A, g, sp)
        c.close()
        print("warmup %d: %d iterations, %.2f s, f = %.12f" % (i, info["iters"], time.perf_counter() - t1,
                                                              info["f"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    iters = []
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        c, info = gpu_eval(ctm, torch, w, A, g, sp)
        iters.append(info["iters"])
        c.close()
        print("step %d: %d iterations" % (i, info["iters"]), file=sys.stderr, flush=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    elapsed = max(ms / 1e3, wall)
    evals_per_s = args.steps / elapsed
    iter_per_s = sum(iters) / elapsed

    roofline = None
    if not args.no_profile_pass:
        print("profile pass" + " (%.0f s)" % (time.perf_counter() - T_START), file=sys.stderr, flush=True)
        c, pinfo = gpu_eval(ctm, torch, w, A, g, sp, profile=True)
        stats = {k: c.kernel_stats(k) for k in KERNEL_CLASSES}
        fac = c.kernel_stats(5)          # the factorisations' share of class 0
        c.close()
        total_ms = sum(v[1] for v in stats.values())
        dom = max((k for k in stats if KERNEL_CLASSES[k][2] is not None), key=lambda k: stats[k][1])
        name, bound, peak = KERNEL_CLASSES[dom]
        launches, kms, kfl, kby = stats[dom]
        ach = kfl / (kms / 1e3) / 1e12 if kms > 0 else None
        roofline = dict(kernel=name, bound=bound, achieved=ach, peak=peak, unit="TFLOP/s",
                        frac=(ach / peak) if ach is not None else None,
                        traffic=measured_traffic(dom),
                        algorithmic_bytes_per_launch=kby / max(launches, 1),
                        algorithmic_flops_per_launch=kfl / max(launches, 1),
                        launches=launches, avg_launch_us=1e3 * kms / max(launches, 1),
                        share_of_kernel_time=kms / total_ms if total_ms > 0 else None,
                        classes={KERNEL_CLASSES[k][0]: dict(launches=v[0], ms=v[1],
                                                            tflops=(v[2] / (v[1] / 1e3) / 1e12) if v[1] > 0 and v[2] > 0 else None)
                                 for k, v in stats.items()})
        # class 0 split into the contraction products (absorption, projector
        # environments, renormalisation, f and g) and the factorisations'
        # products (subspace iteration, Cholesky QR, Rayleigh-Ritz, projector
        # assembly)
        con = tuple(a - b for a, b in zip(stats[0], fac))
        split = {}
        for key, v in (("contraction", con), ("factorisation", fac)):
            tf = v[2] / (v[1] / 1e3) / 1e12 if v[1] > 0 else None
            split[key] = dict(launches=int(v[0]), ms=v[1], flops_per_launch=v[2] / max(v[0], 1),
                              tflops=tf, frac=(tf / PEAK_FP64_MFMA_TFLOPS) if tf is not None else None)
        roofline["fp64_gemm_split"] = split

    fp32 = None
    if not args.no_fp32_leg:
        # reduced-precision form: FP32 products / FP32 accumulation in the bulk
        # contractions, FP64 projectors, spectrum, f and g (same workload)
        print("fp32 leg" + " (%.0f s)" % (time.perf_counter() - T_START), file=sys.stderr, flush=True)
        c, _ = gpu_eval(ctm, torch, w, A, g, sp, precision=ctm.CTM_FP32, refine=True)
        c.close()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        it32 = []
        for i in range(args.steps):
            c, info32 = gpu_eval(ctm, torch, w, A, g, sp, precision=ctm.CTM_FP32, refine=True)
            it32.append(info32["iters"])
            c.close()
        torch.cuda.synchronize()
        el32 = time.perf_counter() - t1
        fp32 = dict(evals_per_s=args.steps / el32, ms_per_step=1e3 * el32 / args.steps,
                    iters_per_eval=float(np.mean(it32)), f=info32["f"],
                    rel_f_vs_fp64=abs(info32["f"] - info["f"]) / abs(info["f"]),
                    speedup_vs_fp64=(args.steps / el32) / evals_per_s)

    reduced = None
    if not args.no_reduced_leg:
        # the reduced method (fused site tensors, C4v CTMRG) on the same
        # workload and the same kernels: the paper's comparison method
        print("reduced-method leg" + " (%.0f s)" % (time.perf_counter() - T_START), file=sys.stderr, flush=True)
        c, _ = gpu_eval(ctm, torch, w, A, g, sp, method="reduced")
        c.close()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        itr = []
        for i in range(args.steps):
            c, infor = gpu_eval(ctm, torch, w, A, g, sp, method="reduced")
            itr.append(infor["iters"])
            c.close()
        torch.cuda.synchronize()
        elr = time.perf_counter() - t1
        reduced = dict(evals_per_s=args.steps / elr, ms_per_step=1e3 * elr / args.steps,
                       iters_per_eval=float(np.mean(itr)), ms_per_iter=1e3 * elr / float(np.sum(itr)),
                       converged=bool(infor["converged"]), f=infor["f"],
                       rel_f_vs_split=abs(infor["f"] - info["f"]) / abs(info["f"]),
                       split_ms_per_iter=1e3 * elapsed / float(np.sum(iters)))
        if not args.no_profile_pass:
            # its GEMM class against the FP64 peak, as for the split path
            c, _ = gpu_eval(ctm, torch, w, A, g, sp, profile=True, method="reduced")
            n_l, kms, kfl, _ = c.kernel_stats(0)
            c.close()
            ach = kfl / (kms / 1e3) / 1e12 if kms > 0 else None
            reduced["gemm"] = dict(launches=n_l, avg_launch_us=1e3 * kms / max(n_l, 1), achieved=ach,
                                   peak=78.6, unit="TFLOP/s", frac=(ach / 78.6) if ach else None)

    lbfgs = None
    if not args.no_lbfgs_leg:
        # the step after the hot path: L-BFGS on f from the workload tensor,
        # every evaluation warm-started from the last converged environments
        from paper_2506_19339_amd import optimize
        print("lbfgs leg" + " (%.0f s)" % (time.perf_counter() - T_START), file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        with optimize.Optimizer(w["beta"], workload_peps(args.workload), w["chi"], env_tol=w["tol"],
                                env_max_iter=w["max_iter"]) as opt:
            r = opt.run(max_steps=args.lbfgs_steps, gtol=1e-7)
        dt = time.perf_counter() - t1
        lbfgs = dict(steps=r.steps, evaluations=r.evaluations, evals_per_s=r.evaluations / dt,
                     moves_per_eval=r.moves / r.evaluations, cold_moves=r.history[0][3],
                     f_start=r.history[0][1], f_end=r.f, g_inf_start=r.history[0][2], g_inf_end=r.g_inf)

    serving = None
    if not args.no_serving_leg:
        # the serving form: the seeded Poisson trace (mean 20 requests/s,
        # beta ~ U[0.18, 0.26], D in {2,3,4,5}, chi in {16,32,64,100,128},
        # f + grad each) replayed in real time with continuous batching
        from paper_2506_19339_amd import serving
        print("serving leg" + " (%.0f s)" % (time.perf_counter() - T_START), file=sys.stderr, flush=True)
        reqs = serving.trace_requests(args.serving_requests, 20.0, 1)
        # each request gets at most SERVING_MAX_ITER moves (a server's work
        # bound per request); one that has not met tol by then is returned
        # flagged (CTM_ENOCONV) and counted in not_converged
        srv = serving.Server(hbm_budget=200 * serving.GiB, max_slots=16, max_iter=SERVING_MAX_ITER)
        done = [0]

        def progress(req):
            done[0] += 1
            if done[0] % 16 == 0:
                print("served %d / %d (%.0f s)" % (done[0], len(reqs), time.perf_counter() - T_START),
                      file=sys.stderr, flush=True)

        st = srv.run(reqs, realtime=True, on_done=progress)
        srv.close()
        serving = st.summary()
        serving["trace"] = ("%d requests, Poisson arrivals at 20/s (seed 1), product state + 0.3 N(0,1) tensors, "
                            "tol 1e-9, max_iter %d" % (len(reqs), SERVING_MAX_ITER))
        serving["failed"] = sum(1 for r in reqs if r.status not in (0, ctm.CTM_ENOCONV))
        serving["not_converged"] = sum(1 for r in reqs if r.status == ctm.CTM_ENOCONV)
        # where the unconverged requests sit: above the simple-cubic Ising
        # critical coupling (0.22165) a symmetric tensor is on the ordered side
        # and its one-site environment need not converge; by bond dimension D
        nc = [r for r in reqs if r.status == ctm.CTM_ENOCONV]
        serving["not_converged_split"] = {
            "beta_above_0.22165": sum(1 for r in nc if r.beta > 0.2216544),
            "beta_below_0.22165": sum(1 for r in nc if r.beta <= 0.2216544),
            "requests_above_0.22165": sum(1 for r in reqs if r.beta > 0.2216544),
            "by_D": {str(D): sum(1 for r in nc if r.D == D) for D in sorted({r.D for r in reqs})}}
        serving["failures"] = ["request %d (D=%d, chi=%d, beta=%.4f): %s" % (r.rid, r.D, r.chi, r.beta, r.error)
                               for r in reqs if r.status not in (0, ctm.CTM_ENOCONV)]

    cpu = None
    if not args.no_cpu_baseline:
        print("cpu baseline (oracle)" + " (%.0f s)" % (time.perf_counter() - T_START), file=sys.stderr, flush=True)
        t3, t2 = cpu_baseline(args.workload, args.cpu_sample_iters)
        n_it = float(np.mean(iters))
        t_eval = n_it * (t3 + t2)
        cpu = dict(value=1.0 / t_eval, unit="evals/s", cores=len(os.sched_getaffinity(0)),
                   kind="oracle",
                   sample="%d steady-state split-CTMRG iterations per network of the same "
                          "workload (after the growth move), %.2f s triple + %.2f s double per "
                          "iteration, extrapolated to %.1f iterations per evaluation"
                          % (args.cpu_sample_iters, t3, t2, n_it))

    out = {
        "metric": "f+grad evals/s (D=5, chi=100, beta=0.22, FP64)",
        "value": evals_per_s,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "%s: beta=%g D=%d chi=%d tol=%g max_iter=%d, A = D4-projected "
                               "N(0,1) tensor (seed %d), f + grad per step"
                               % (args.workload, w["beta"], w["D"], w["chi"], w["tol"],
                                  w["max_iter"], w["seed"])},
        "ctmrg_iter_per_s": iter_per_s,
        "iters_per_eval": float(np.mean(iters)),
        "f": info["f"],
        "roofline": roofline,
        "fp32_form": fp32,
        "reduced_method": reduced,
        "lbfgs": lbfgs,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
