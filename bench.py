"""Benchmark of the restarted-PDHG LP solver on one MI355X.

Workload: the large skewed random LP (m = 1e6 rows, half EQ and half LE,
n = 2e6 variables in [0, 10], nnz = 2e7 with power-law row lengths capped at
10,000, N(0,1) values, constructed optimum), FP64 matrix.

A "step" is one accepted PDHG iteration of Algorithm 1 (both fused SpMV step
kernels plus the amortised restart/termination evaluation every 64 steps),
timed inside pdlp_solve with the iterate already resident in HBM.  The line
also carries:
  roofline     -- the dominant step kernel's algorithmic bytes per launch over
                  its mean launch duration (HIP events on the solver's stream),
                  against 8 TB/s, and the fixed cost of a solve without steps;
  roofline_fp32_matrix -- the same for both step kernels with the FP32 matrix;
  cpu_baseline -- the FP64 CPU oracle on the same LP on the host cores: a solve
                  to rel KKT 1e-4 with every core (capped, never extrapolated)
                  and the first iterations with one thread;
  time_to_tol  -- wall time to rel KKT 1e-4 with the FP64 and the FP32 matrix and to
                  1e-8 with the FP64 matrix, and of the 2000 x 2000 transportation LP to 1e-6;
  small_lp     -- the m = 1000, n = 2000 random LP to 1e-4 and 1e-8, GPU and oracle;
  batch, warm_start -- the 4,096-LP batch and the learned warm start.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# the step kernels and the sources that lay out what they read (row order,
# row blocks, column panels)
STEP_SOURCES = ("pdlp_dev.h", "pdlp_ops.h", "kernels.hip", "setup.hip", "pdlp_api.cpp")


def _code_only(text: str) -> str:
    """C++ source without its comments and blank lines (string literals here
    hold no comment markers), so that a comment edit keeps the hash."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def step_kernels_hash() -> str:
    """sha256 prefix over the code (comments dropped) of the sources the
    single-LP step kernels and their matrix layout are built from."""
    import hashlib
    h = hashlib.sha256()
    for name in STEP_SOURCES:
        h.update(_code_only(open(os.path.join(ROOT, "paper_2311_12180_amd", "csrc", name)).read()).encode())
    return h.hexdigest()[:16]


def _traffic_from_profiles(kernel: str):
    """Bytes between L2 and the memory fabric per launch of step `kernel`
    (primal_step / dual_step) from the committed rocprofv3 counter summary
    (lines 'step <name> fetch_bytes <F> write_bytes <W>'), or None when there is
    none or it was taken from different step-kernel or layout sources (the
    summary records the sha256 prefix of STEP_SOURCES)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "step_kernels_skewed_1e6x2e6_traffic.txt")
    if not os.path.exists(path):
        return None
    cur = step_kernels_hash()
    text = open(path).read()
    if f"sha256[:16] = {cur}" not in text:
        return None
    for line in text.splitlines():
        parts = line.split()
        if len(parts) >= 6 and parts[0] == "step" and parts[1] == kernel:
            return float(parts[3]) + float(parts[5])
    return None


def host_threads() -> int:
    cores = len(os.sched_getaffinity(0))
    env_threads = os.environ.get("OMP_NUM_THREADS")
    return min(cores, int(env_threads)) if env_threads and env_threads.isdigit() else cores


def cpu_baseline(prob, eps: float, cap_s: float, iters_1t: int):
    """The oracle on the 1e6 x 2e6 LP on the host cores: with every core, a
    solve to rel KKT eps capped at cap_s seconds of solve time (never
    extrapolated), whose iterations per second are the baseline value; with
    one thread, the first iters_1t accepted iterations."""
    import oracle
    oracle.build()
    threads = host_threads()
    t0 = time.time()
    r = oracle.solve(prob, eps_rel=eps, max_iter=1_000_000, time_limit_s=cap_s, threads=threads)
    wall = time.time() - t0
    info = r.info
    reached = r.status == "OPTIMAL"
    t1 = time.time()
    r1 = oracle.solve(prob, eps_rel=0.0, max_iter=iters_1t, threads=1)
    wall1 = time.time() - t1
    i1 = r1.info
    return {"value": info["iterations"] / info["solve_s"], "unit": "PDHG iters/sec", "cores": info["threads_used"],
            "kind": "oracle",
            "sample": (f"a solve of the same 1e6x2e6 LP (FP64) to rel KKT {eps:g}, capped at {cap_s:g} s: "
                       f"{info['iterations']} accepted iterations ({info['attempts']} attempts, "
                       f"{info['evaluations']} evaluations) in {info['solve_s']:.1f} s, "
                       + ("tolerance reached" if reached else f"not reached in {info['solve_s']:.1f} s")
                       + f"; setup {info['setup_s']:.1f} s excluded, total {wall:.1f} s"),
            "time_to_tol_s": round(info["solve_s"], 2) if reached else None,
            "status": r.status, "primal_obj": info["primal_obj"],
            "one_thread": {"value": i1["iterations"] / i1["solve_s"], "cores": i1["threads_used"],
                           "sample": f"first {i1['iterations']} accepted iterations in {i1['solve_s']:.1f} s "
                                     f"(setup {i1['setup_s']:.1f} s excluded, total {wall1:.1f} s)"}}


def small_lp_section(P, stream, seeds=(0, 1, 2)):
    """The m = 1000, n = 2000 random LP (8 nonzeros per column) to rel KKT
    1e-4 and 1e-8: GPU wall time (setup and solve apart) and iterations per
    second, the attempt-slot floor, and the oracle with every host core and
    with one thread on the same LPs; objective error of the GPU's solution
    against the oracle's."""
    import lpgen
    import oracle
    oracle.build()
    out = {"workload": "random LP m=1000 (500 EQ, 500 LE), n=2000, 8 nnz per column, x in [0,10], FP64",
           "seeds": list(seeds)}
    for eps in (1e-4, 1e-8):
        g_solve, g_setup, g_it, g_att, errs = [], [], [], [], []
        o_all, o_one, o_it = [], [], []
        for sd in seeds:
            p = lpgen.config0(sd)
            h = P.pdlp_create(p, stream=stream, eps_rel=eps, time_limit_s=60.0)
            P.pdlp_solve(h)          # first solve: graph capture, code load
            P.pdlp_solve(h)
            _, _, _, inf = P.pdlp_get_solution(h)
            P.pdlp_destroy(h)
            r = oracle.solve(p, eps_rel=eps, threads=host_threads())
            r1 = oracle.solve(p, eps_rel=eps, threads=1)
            g_solve.append(inf["solve_s"]); g_setup.append(inf["setup_s"])
            g_it.append(inf["iterations"]); g_att.append(inf["attempts"])
            o_all.append(r.info["solve_s"]); o_one.append(r1.info["solve_s"]); o_it.append(r.info["iterations"])
            ro = r.info["primal_obj"]
            errs.append(abs(inf["primal_obj"] - ro) / (1 + abs(ro)))
        out[f"{eps:g}"] = {
            "gpu_solve_s": [round(v, 4) for v in g_solve], "gpu_setup_s": [round(v, 4) for v in g_setup],
            "gpu_iterations": g_it, "gpu_attempts": g_att,
            "gpu_iters_per_s": round(float(np.sum(g_it) / np.sum(g_solve)), 1),
            "gpu_attempts_per_s": round(float(np.sum(g_att) / np.sum(g_solve)), 1),
            "oracle_solve_s_all_cores": [round(v, 4) for v in o_all],
            "oracle_solve_s_one_thread": [round(v, 4) for v in o_one],
            "oracle_iterations": o_it, "oracle_cores": host_threads(),
            "oracle_iters_per_s_all_cores": round(float(np.sum(o_it) / np.sum(o_all)), 1),
            "oracle_iters_per_s_one_thread": round(float(np.sum(o_it) / np.sum(o_one)), 1),
            "obj_rel_err_vs_oracle_max": max(errs)}
        log(f"random 1000x2000 to {eps:g}: {out[f'{eps:g}']}")
    return out


def _gen_batch_lp(args):
    import lpgen
    seed, i, m = args
    return lpgen.batch_lp(seed, i, m)


def _oracle_one(args):
    import oracle
    p, eps = args
    r = oracle.solve(p, eps_rel=eps, max_iter=200000, threads=1)
    return r.info["primal_obj"], r.info["iterations"], r.info["solve_s"], r.status


def batch_section(P, stream, count: int, eps: float, sample: int):
    """4096 random LPs (m ~ U{50..2000}, n = 2m, 8 nnz per column) solved in
    one persistent launch to rel KKT eps, against the same LPs solved one by
    one with the single-LP path (a sample) and the oracle (a sample, one LP
    per host thread)."""
    import lpgen
    import oracle
    from concurrent.futures import ProcessPoolExecutor
    oracle.build()
    ms = lpgen.batch_sizes(0, 4096)[:count]
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    t = time.time()
    with ProcessPoolExecutor(workers) as ex:
        probs = list(ex.map(_gen_batch_lp, [(0, i, int(ms[i])) for i in range(count)], chunksize=16))
    log(f"batch: generated {count} LPs in {time.time() - t:.1f}s ({workers} processes)")
    t = time.time()
    h = P.pdlp_create_batch(probs, stream=stream, eps_rel=eps, max_iter=200000, time_limit_s=600.0)
    create_s = time.time() - t
    lanes, grid = P.pdlp_batch_schedule(h)
    P.pdlp_solve_batch(h)          # first solve: code load, caches
    t = time.perf_counter()
    P.pdlp_solve_batch(h)
    solve_s = time.perf_counter() - t
    x, y, rc, infos = P.pdlp_get_solution_batch(h, -1)
    its = np.array([i["iterations"] for i in infos], np.int64)
    att = np.array([i["attempts"] for i in infos], np.int64)
    ev = np.array([i["evaluations"] for i in infos], np.int64)
    status = [i["status_name"] for i in infos]
    handed = int(sum(1 for i in infos if i["handoff_k"] > 0))
    nnz = np.array([p.nnz for p in probs], np.float64)
    mm = np.array([p.m for p in probs], np.float64)
    nn = np.array([p.n for p in probs], np.float64)
    # algorithmic bytes: each attempt streams K~' and K~ once (values + column
    # indices + row pointers), reads/writes the step vectors; each evaluation
    # runs three products with two gathered vectors plus the vector passes
    att_bytes = att * (2 * nnz * 12 + 4 * (mm + nn) + 72 * nn + 69 * mm)
    ev_bytes = ev * (3 * nnz * 12 + 2 * 4 * (mm + nn) + 16 * (mm + nn) + 120 * nn + 100 * mm)
    gbps = float((att_bytes.sum() + ev_bytes.sum()) / solve_s / 1e9)
    # the same LPs one by one through the single-LP path (sample)
    t = time.perf_counter()
    single_its = []
    for k in range(sample):
        hs = P.pdlp_create(probs[k], stream=stream, eps_rel=eps, max_iter=200000, time_limit_s=60.0)
        P.pdlp_solve(hs)
        single_its.append(P.pdlp_get_solution(hs)[3]["iterations"])
        P.pdlp_destroy(hs)
    single_s = (time.perf_counter() - t) / sample
    # oracle on a sample, one LP per host thread
    t = time.time()
    with ProcessPoolExecutor(workers) as ex:
        orc = list(ex.map(_oracle_one, [(probs[k], eps) for k in range(sample)]))
    orc_wall = time.time() - t
    obj_err = max(abs(infos[k]["primal_obj"] - orc[k][0]) / (1 + abs(orc[k][0])) for k in range(sample))
    recheck = max(oracle.evaluate(probs[k], x[h.col_off[k]:h.col_off[k + 1]],
                                  y[h.row_off[k]:h.row_off[k + 1]])["rel_kkt"] for k in range(sample))
    P.pdlp_destroy(h)
    u, cnt = np.unique(lanes, axis=0, return_counts=True)
    return {"workload": f"{count} random LPs, m ~ U{{50..2000}} (half EQ, half LE), n = 2m, 8 nnz per column, "
                        f"rel KKT {eps:g}, FP64",
            "lps": count, "nnz_total": int(nnz.sum()), "create_s": round(create_s, 3),
            "solve_s": round(solve_s, 4), "lps_per_s": round(count / solve_s, 1),
            "optimal": status.count("OPTIMAL"), "iterations_mean": float(its.mean()), "iterations_max": int(its.max()),
            "lp_iters_per_s": round(float(its.sum() / solve_s), 1),
            "handed_off": {"after_steps": 2048, "streams": 8, "lps": handed},
            "algorithmic_GBps": round(gbps, 1), "frac_of_hbm_peak": round(gbps / PEAK_HBM_GBPS, 4),
            "schedule": {"grid": int(grid), "lanes_k_kt_counts": [[int(a), int(b), int(c)]
                                                                 for (a, b), c in zip(u.tolist(), cnt.tolist())]},
            "single_lp_path": {"sample": sample, "s_per_lp": round(single_s, 5),
                               "lps_per_s": round(1.0 / single_s, 1),
                               "batch_speedup": round((count / solve_s) * single_s, 2)},
            "cpu_baseline": {"kind": "oracle", "sample": sample, "cores": workers,
                             "lps_per_s": round(sample / orc_wall, 2),
                       "obj_rel_err_max_vs_gpu": obj_err, "gpu_rel_kkt_cpu_recheck_max": recheck}}


def _gen_family_lp(args):
    import lpgen
    seed, i = args
    return lpgen.transport_family_lp(seed, i, 100, 100)


def warmstart_section(P, stream, n_train: int, n_test: int, epochs: int, batch: int, lr: float, eps: float):
    """Learned warm start on a family of 100 x 100 transportation LPs: cold
    batched solves give the targets, the network trains on the GPU, and the
    held-out LPs are solved warm (cold fallback) and cold to rel KKT eps."""
    import lpgen
    from concurrent.futures import ProcessPoolExecutor
    from paper_2311_12180_amd import gnn as G
    from paper_2311_12180_amd import warmstart as W
    count = n_train + n_test
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    t = time.time()
    with ProcessPoolExecutor(workers) as ex:
        probs = list(ex.map(_gen_family_lp, [(0, i) for i in range(count)], chunksize=64))
    gen_s = time.time() - t
    log(f"warm start: generated {count} LPs in {gen_s:.1f}s")
    # targets: cold solves of the training LPs (one batched launch)
    xs, ys, infos, cold_train_s = W.solve_batch(probs[:n_train], eps, stream)
    ok = [k for k, i in enumerate(infos) if i["status_name"] == "OPTIMAL"]
    ys = [W.canonical_transport_duals(y, 100) for y in ys]
    om = np.array([infos[k]["omega"] for k in range(n_train)])
    log(f"warm start: cold solves of {n_train} training LPs in {cold_train_s:.1f}s ({len(ok)} optimal)")
    train_probs = [probs[k] for k in ok]
    gs = G.pdlp_gnn_create(train_probs, [xs[k] for k in ok], [ys[k] for k in ok], om[ok], stream=stream)
    theta0 = lpgen.gnn_init(0, _gnn_shapes())
    # unit-scale loss terms: targets in the network's units (x s_a/s_b, y s_a/s_c; s_a = 1 here)
    sb = [float(np.max(np.abs(probs[k].b))) for k in ok]
    sc = [float(np.max(np.abs(probs[k].c))) for k in ok]
    wts = W.balance_weights([xs[k] / sb[i] for i, k in enumerate(ok)], [ys[k] / sc[i] for i, k in enumerate(ok)],
                            np.log(om[ok]))
    losses, train_s = W.train(gs, len(ok), epochs, batch, lr, theta0, seed=0, log=log, weights=wts)
    theta = G.pdlp_gnn_get_params(gs)
    G.pdlp_gnn_destroy(gs)
    # held-out LPs: predict, warm solve (with fallback), cold solve
    test = probs[n_train:]
    gt = G.pdlp_gnn_create(test, stream=stream)
    G.pdlp_gnn_set_params(gt, theta)
    t = time.perf_counter()
    x0, y0, om0 = W.predict(gt, 0, n_test)
    infer_s = time.perf_counter() - t
    G.pdlp_gnn_destroy(gt)
    _, _, cold, cold_s = W.solve_batch(test, eps, stream)
    warm, warm_s, fb_s, fb = W.warm_solve_with_fallback(test, eps, (x0, y0, om0), stream)
    ci = np.array([i["iterations"] for i in cold], float)
    wi = np.array([i["iterations"] for i in warm], float)
    # the same held-out LPs warm-started from the mean training solution (no network)
    xm = np.mean([xs[k] for k in ok], axis=0)
    ym = np.mean([ys[k] for k in ok], axis=0)
    _, _, avg, avg_s = W.solve_batch(test, eps, stream, warm=([xm] * n_test, [ym] * n_test,
                                                             np.full(n_test, float(np.exp(np.mean(np.log(om[ok])))))))
    ai = np.array([i["iterations"] for i in avg], float)
    return {"workload": f"{count} transportation LPs 100 x 100 (n = 10,000, m = 200) of one family; "
                        f"train {n_train}, test {n_test}; rel KKT {eps:g}",
            "generate_s": round(gen_s, 1), "cold_train_solves_s": round(cold_train_s, 2),
            "train": {"epochs": epochs, "batch_lps": batch, "lr": lr, "seconds": round(train_s, 2),
                      "loss_weights": [round(w, 4) for w in wts],
                      "loss_first_epoch": losses[0], "loss_last_epoch": losses[-1]},
            "inference_s": round(infer_s, 4),
            "test_cold": {"solve_s": round(cold_s, 3), "iterations_mean": float(ci.mean()),
                          "iterations_median": float(np.median(ci)), "optimal": sum(i["status_name"] == "OPTIMAL" for i in cold)},
            "test_warm": {"solve_s": round(warm_s, 3), "fallback_s": round(fb_s, 3), "fallbacks": len(fb),
                          "iterations_mean": float(wi.mean()), "iterations_median": float(np.median(wi)),
                          "optimal": sum(i["status_name"] == "OPTIMAL" for i in warm)},
            "test_warm_from_mean_solution": {"solve_s": round(avg_s, 3), "iterations_mean": float(ai.mean())},
            "iterations_ratio_warm_over_cold": round(float(wi.mean() / ci.mean()), 4),
            "time_ratio_warm_over_cold": round(float((warm_s + fb_s + infer_s) / cold_s), 4)}


def _gnn_shapes():
    H = 64
    shapes = [("W_v0", (5, H)), ("b_v0", (H,)), ("W_c0", (4, H)), ("b_c0", (H,))]
    for r in range(3):
        shapes += [(f"Phi{r}", (2 * H, H)), (f"phi{r}", (H,)), (f"Psi{r}", (2 * H, H)), (f"psi{r}", (H,))]
    return shapes + [("w_x", (H,)), ("b_x", (1,)), ("w_y", (H,)), ("b_y", (1,)), ("w_o", (2 * H,)), ("b_o", (1,))]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-ttt", action="store_true", help="skip the time-to-tolerance solves")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-cap", type=float, default=60.0,
                    help="solve-time cap (s) of the all-core oracle run to rel KKT 1e-4 on the large LP")
    ap.add_argument("--cpu-iters-1t", type=int, default=16,
                    help="accepted iterations of the one-thread oracle sample on the large LP")
    ap.add_argument("--no-small", action="store_true", help="skip the m=1000, n=2000 random LP section")
    ap.add_argument("--only", choices=("small", "batch", "warmstart"),
                    help="run only that section and print its JSON (for profiling)")
    ap.add_argument("--ttt-limit", type=float, default=90.0)
    ap.add_argument("--profile-attempts", type=int, default=200)
    ap.add_argument("--layout", type=int, nargs=2, default=(-1, -2), metavar=("K", "KT"),
                    help="SpMV layouts of K and K' (-1: chosen at create by timing; pin them for profiler runs)")
    ap.add_argument("--detect-infeas", type=int, default=1, choices=(0, 1),
                    help="infeasibility certificates at every evaluation (the library default is on)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-LP section")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--batch-sample", type=int, default=64)
    ap.add_argument("--no-warmstart", action="store_true", help="skip the learned warm-start section")
    ap.add_argument("--ws-train", type=int, default=16000)
    ap.add_argument("--ws-test", type=int, default=4000)
    ap.add_argument("--ws-epochs", type=int, default=10)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the solver does not shard "
              "an LP over several GPUs", file=sys.stderr)
        sys.exit(2)

    import torch
    import lpgen
    from paper_2311_12180_amd import pdlp as P

    assert torch.cuda.is_available(), "needs a ROCm GPU"
    dev = torch.device("cuda:0")
    if args.only:
        st = torch.cuda.current_stream().cuda_stream
        if args.only == "small":
            out = small_lp_section(P, st)
        elif args.only == "batch":
            out = batch_section(P, st, args.batch_count, 1e-6, args.batch_sample)
        else:
            out = warmstart_section(P, st, args.ws_train, args.ws_test, args.ws_epochs, 64, 1e-3, 1e-6)
        print(json.dumps(out), flush=True)
        return
    t = time.time()
    prob = lpgen.config1(0)
    log(f"generated {prob.name} in {time.time() - t:.1f}s")

    # device copy bandwidth (context for the roofline)
    a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a); torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record(); torch.cuda.synchronize()
    copy_gbps = 10 * 2 * a.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b

    stream = torch.cuda.current_stream().cuda_stream
    h = P.pdlp_create(prob, stream=stream, eps_rel=0.0, max_iter=args.warmup, time_limit_s=600.0,
                      spmv_layout=args.layout[0], spmv_layout_kt=args.layout[1], detect_infeas=args.detect_infeas)
    _, _, _, info0 = None, None, None, None
    P.pdlp_solve(h)            # warm-up: graph capture, first launches
    log(f"setup {P.pdlp_get_solution(h)[3]['setup_s']:.2f}s; warm-up {args.warmup} steps done")
    P.pdlp_set_termination(h, 0.0, args.steps, 600.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.pdlp_solve(h)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _, _, _, info = P.pdlp_get_solution(h)
    steps = int(info["iterations"])
    assert steps == args.steps, info
    ms_step = dt / steps * 1e3
    log(f"timed {steps} steps in {dt:.3f}s: {steps / dt:.1f} it/s ({info['attempts']} attempts, "
        f"{info['restarts']} restarts)")

    # per-kernel durations (HIP events on the solver's stream) and the roofline
    ms_a, ms_b = P.pdlp_profile_attempts(h, args.profile_attempts)
    by_a, by_b = P.pdlp_step_bytes(h)
    # a step is one kernel (row blocks, SELL-64 chunks) or two (column panels: segment sums, then
    # rows; LDS-staged panels: the long rows' panel segment sums, then the row pass)
    names = {0: "{}<{}>", 1: "k_seg<{1}> + k_rows<{1}>", 2: "{}<{}> (XCD-contiguous blocks)",
             3: "k_stage<{1}> + k_stage_rows<{1}> (LDS-staged panels)"}
    lk, lt = info["layout_k"], info["layout_kt"]

    def kname(lay, op):
        if lay & 64:
            cfg = (lay >> 4) & 3
            return (f"k_sell<{op}> (SELL-64 chunks, " +
                    ("256-thread workgroups)" if cfg == 2 else f"{1024 >> cfg}-thread workgroups, LDS slice of y)"))
        if (lay & 3) == 3:
            return names[3].format("", op) + f" ({256 << (lay >> 4)}-thread staging workgroups)"
        return (names[lay & 3].format("k_fused", op) + (" (persistent grid)" if lay & 4 else "") +
                (" (6144-nonzero blocks)" if lay & 8 else ""))
    kern = {"primal_step": (ms_a, by_a, kname(lt, "PrimalOp")), "dual_step": (ms_b, by_b, kname(lk, "DualOp"))}
    dom = max(kern, key=lambda k: kern[k][0])
    ms_d, by_d, kname = kern[dom]
    achieved = by_d / (ms_d * 1e-3) / 1e9
    traffic = _traffic_from_profiles(dom)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": traffic, "kernel": f"{dom}: {kname}",
                "bytes_per_launch": by_d, "ms_per_launch": ms_d,
                "other_kernel": {"name": [k for k in kern if k != dom][0],
                                 "ms_per_launch": kern[[k for k in kern if k != dom][0]][0],
                                 "GBps": round(kern[[k for k in kern if k != dom][0]][1] /
                                               (kern[[k for k in kern if k != dom][0]][0] * 1e-3) / 1e9, 1)},
                "copy_GBps": round(copy_gbps, 1)}
    # fixed cost of a solve: the starting evaluation, the output and the
    # host-device round trips, without any step (max_iter = 0)
    P.pdlp_set_termination(h, 0.0, 0, 600.0)
    fixed = []
    for _ in range(5):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        P.pdlp_solve(h)
        torch.cuda.synchronize()
        fixed.append(time.perf_counter() - t1)
    roofline["solve_fixed_ms"] = round(1e3 * float(np.median(fixed)), 3)
    log(f"roofline: {roofline}")
    P.pdlp_destroy(h)

    # the same step kernels with the FP32 matrix (FP64 accumulation and iterates)
    h = P.pdlp_create(prob, stream=stream, eps_rel=0.0, max_iter=args.warmup, time_limit_s=600.0,
                      a_precision=1, detect_infeas=args.detect_infeas)
    P.pdlp_solve(h)
    ms_a32, ms_b32 = P.pdlp_profile_attempts(h, args.profile_attempts)
    by_a32, by_b32 = P.pdlp_step_bytes(h)
    i32 = P.pdlp_get_solution(h)[3]
    roof32 = {"layout_k_kt": [i32["layout_k"], i32["layout_kt"]]}
    for nm, ms_, by_ in (("primal_step", ms_a32, by_a32), ("dual_step", ms_b32, by_b32)):
        ach = by_ / (ms_ * 1e-3) / 1e9
        roof32[nm] = {"bytes_per_launch": by_, "ms_per_launch": ms_, "achieved": round(ach, 1),
                      "frac": round(ach / PEAK_HBM_GBPS, 4)}
    roof32["ms_per_attempt_pair"] = round(ms_a32 + ms_b32, 4)
    roof32["fp64_ms_per_attempt_pair"] = round(ms_a + ms_b, 4)
    log(f"roofline, FP32 matrix: {roof32}")
    P.pdlp_destroy(h)

    ttt = None
    if not args.no_ttt:
        ttt = {}
        import oracle
        oracle.build()
        # (name, matrix precision, tolerance, presolve, restart metric: 0 KKT, 1 normalized duality gap)
        runs = [("fp64_1e-4", 0, 1e-4, 0, 0), ("fp32_matrix_1e-4", 1, 1e-4, 0, 0), ("fp64_1e-8", 0, 1e-8, 0, 0),
                ("fp64_presolve_1e-4", 0, 1e-4, 1, 0), ("fp64_presolve_1e-8", 0, 1e-8, 1, 0),
                ("fp64_gap_restarts_1e-4", 0, 1e-4, 0, 1)]
        for name, prec, eps, pre, metric in runs:
            h = P.pdlp_create(prob, stream=stream, eps_rel=eps, a_precision=prec, time_limit_s=args.ttt_limit,
                              presolve=pre, restart_metric=metric)
            P.pdlp_solve(h)
            x, y, rc, inf = P.pdlp_get_solution(h)
            ev = oracle.evaluate(prob, x, y)
            obj_star = prob.obj_star()
            ttt[name] = {"status": inf["status_name"], "iterations": inf["iterations"],
                         "attempts": inf["attempts"], "restarts": inf["restarts"],
                         "setup_s": round(inf["setup_s"], 3), "solve_s": round(inf["solve_s"], 3),
                         "iters_per_s": round(inf["iterations"] / max(inf["solve_s"], 1e-9), 1),
                         "rel_kkt_gpu": inf["rel_kkt"], "rel_kkt_cpu_fp64_recheck": ev["rel_kkt"],
                         "primal_obj": inf["primal_obj"],
                         "obj_rel_err_vs_known_optimum": abs(inf["primal_obj"] - obj_star) / (1 + abs(obj_star))}
            if pre:
                ttt[name]["solved_m_n"] = [inf["m_solved"], inf["n_solved"]]
            log(f"time to {eps:g} ({name}): {ttt[name]}")
            P.pdlp_destroy(h)
        # the 2000 x 2000 transportation LP (n = 4e6, m = 4000, nnz = 8e6) to 1e-6, both restart metrics
        import lpgen
        tp = lpgen.config2(0)
        for name, metric in (("transport_2000x2000_1e-6", 0), ("transport_2000x2000_gap_restarts_1e-6", 1)):
            h = P.pdlp_create(tp, stream=stream, eps_rel=1e-6, time_limit_s=args.ttt_limit, restart_metric=metric)
            P.pdlp_solve(h)
            x, y, rc, inf = P.pdlp_get_solution(h)
            ev = oracle.evaluate(tp, x, y)
            ttt[name] = {
                "status": inf["status_name"], "iterations": inf["iterations"], "attempts": inf["attempts"],
                "restarts": inf["restarts"], "setup_s": round(inf["setup_s"], 3), "solve_s": round(inf["solve_s"], 3),
                "iters_per_s": round(inf["iterations"] / max(inf["solve_s"], 1e-9), 1),
                "rel_kkt_gpu": inf["rel_kkt"], "rel_kkt_cpu_fp64_recheck": ev["rel_kkt"],
                "primal_obj": inf["primal_obj"], "layout_k_kt": [inf["layout_k"], inf["layout_kt"]]}
            log(f"transportation to 1e-6 ({name}): {ttt[name]}")
            P.pdlp_destroy(h)

    batch = None
    if not args.no_batch:
        batch = batch_section(P, stream, args.batch_count, 1e-6, args.batch_sample)
        log(f"batch: {batch}")

    ws = None
    if not args.no_warmstart:
        ws = warmstart_section(P, stream, args.ws_train, args.ws_test, args.ws_epochs, 64, 1e-3, 1e-6)
        log(f"warm start: {ws}")

    small = None
    if not args.no_small:
        small = small_lp_section(P, stream)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(prob, 1e-4, args.cpu_cap, args.cpu_iters_1t)
        log(f"cpu baseline: {cpu}")
        if ttt is not None:
            # each GPU objective at rel KKT 1e-4 against the FP64 oracle's objective at the same tolerance
            ro = cpu["primal_obj"]
            for name in ("fp64_1e-4", "fp32_matrix_1e-4"):
                if cpu["status"] == "OPTIMAL":
                    ttt[name]["obj_rel_err_vs_oracle_1e-4"] = abs(ttt[name]["primal_obj"] - ro) / (1 + abs(ro))

    line = {"metric": "PDHG iters/sec + wall time to rel KKT 1e-4/1e-8; SpMV HBM GB/s vs peak",
            "value": round(steps / dt, 2), "unit": "PDHG iters/sec", "n_gpus": 1, "steps": steps,
            "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "skewed random LP m=1e6 (half EQ, half LE) n=2e6 nnz=2e7, row lengths "
                                   "power-law capped at 10,000, FP64 matrix",
                       "m": prob.m, "n": prob.n, "nnz": prob.nnz, "eval_period": 64,
                       "spmv_layout_k_kt": [info["layout_k"], info["layout_kt"]]},
            "roofline": roofline, "roofline_fp32_matrix": roof32, "cpu_baseline": cpu, "time_to_tol": ttt,
            "small_lp": small, "batch": batch, "warm_start": ws}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
