"""Benchmark: batched forward + adjoint rollouts on one MI355X.

A step is one pass of the whole hot path over one batch: dmx_rollout (adaptive
Dormand-Prince 5(4) with the soft-contact Newton solve, tape of accepted steps)
followed by dmx_rollout_vjp (discrete adjoint of the summed final position),
on the cube-on-plane workload: 4096 free cubes (edge 0.2 m, 1 kg) with 8
corner-sphere contacts, stiff contact (t_c 1 ms), random pose and velocity,
0.5 s horizon, rtol 1e-6, atol 1e-8, FP64 throughout.

Prints one JSON line with the throughput in world-simulated seconds per wall
second, the roofline of the dominant kernel (FP64 ALU bound, algorithmic
FLOPs from per-unit counts x work units counted by the kernels), the plain
one-world-per-launch GPU form of the same kernels, and the CPU oracle timed on
this host.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X vector FP64 (256 CUs x 2.4 GHz x 128 flop/clk)
PEAK_HBM_GBS = 8000.0

# Algorithmic FP64 operations per counted work unit of the free-body kernels
# (FMA = 2; divisions, square roots and transcendental calls = 1), counted
# from the operations each unit must perform; nc = contact slots of the model.
FWD_FLOPS = {
    "attempts": 1450,          # 6 stage combinations, 7 (+)-maps, error estimate, controller
    "rhs": (93, 38),           # frame, bias, a0 (93) + slot geometry per slot (38 * nc)
    "rhs_contacts": 190,       # rows of an active contact (J_n, J_t, impedance, a_ref) + activity test
    "newton_iters": 204,       # M terms, 6x6 Cholesky, two triangular solves, step update
    "newton_contacts": 113,    # directional data, team sums, activity re-test per active contact
    "newton_edges": 85,        # gradient (25) and Hessian (60) contribution per active edge
    "ls_contacts": 40,         # line-search piece test per contact and iteration
}
ADJ_FLOPS = {
    "steps": 2500,             # 7 stage rebuilds and cotangent distribution through (+) and the tableau
    "vjps": (557, 38),         # frame, Hessian assembly, Cholesky, solve, bias and quaternion VJPs + slots
    "vjp_contacts": 490,       # rows, activity, geometry and frame cotangents per active contact
    "vjp_edges": 160,          # Hessian term and implicit-solution cotangents per active edge
}


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    if it was taken on the kernels as built now (same device-code digest)."""
    import re
    from paper_2506_14186_amd import build as B
    path = os.path.join(ROOT, "profiles", "hbm_traffic_cube_toss_4096.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    dig = re.search(r"^kernel-digest: (\w+)", text, re.M)
    val = re.search(rf"^traffic-bytes {kernel}: (\d+)", text, re.M)
    if not dig or not val or dig.group(1) != B.kernel_digest():
        return None
    return int(val.group(1))


def algorithmic_flops(counters, table, nc):
    total = 0.0
    for name, per in table.items():
        n = float(counters[name])
        if isinstance(per, tuple):
            total += n * (per[0] + per[1] * nc)
        else:
            total += n * per
    return total


def serve_leg(D, W, rate, seconds, seed=5, drain_s=240.0):
    """MPC requests arriving as a Poisson stream: each picks the controlled
    corner-sphere cube, the legged chain or the box-geom cube (the one-level
    stack), N ~ U{16..256} candidate control sequences
    u ~ U(-1, 1) over H ~ U{50..500} intervals of 10 ms, and asks for the
    candidates' costs and control gradients.  Latency = completion - arrival
    (submission happens at the arrival time)."""
    rng = np.random.default_rng(seed)
    models = {"cube": D.Model(W.model_cube_corners(ctrl=True)), "chain": D.Model(W.model_chain()),
              "box": D.Model(W.model_box(ctrl=True, mu=0.6, tc=0.003))}
    chain_x0 = W.chain_walk(n_worlds=1, n_intervals=1)["x0"][0]
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=int(rate * seconds * 2) + 16))
    arrivals = arrivals[arrivals < seconds]
    srv = D.Server(hbm_budget_bytes=200 * 10 ** 9, max_batch_worlds=16384)
    pending, lat, done_kinds, work = {}, [], [], 0.0
    t0 = time.perf_counter()
    nxt = 0
    backlog_at_end = None
    t_last = t0
    try:
        while nxt < len(arrivals) or pending:
            now = time.perf_counter() - t0
            while nxt < len(arrivals) and arrivals[nxt] <= now:
                kind = ("cube", "chain", "box")[int(rng.integers(3))]
                m = models[kind]
                N, H = int(rng.integers(16, 257)), int(rng.integers(50, 501))
                if kind == "cube":
                    x0 = W.cube_toss(seed=int(rng.integers(1 << 30)), n_worlds=1, horizon=0.1)["x0"][0]
                elif kind == "box":
                    x0 = W.box_toss(seed=int(rng.integers(1 << 30)), n_worlds=1, horizon=0.1)["x0"][0]
                else:
                    x0 = chain_x0
                u = rng.uniform(-1.0, 1.0, size=(N, H, m.nu))
                target = [float(rng.normal(0, 0.2)), float(rng.normal(0, 0.2)), 0.3]
                pending[srv.submit(m, x0, u, 0.01, target, ctrl_weight=1e-3)] = (arrivals[nxt], kind, N * H * 0.01)
                nxt += 1
            if backlog_at_end is None and now >= seconds:
                backlog_at_end = len(pending)
            for t in list(pending):
                r = srv.poll(t)
                if r is not None:
                    arr, kind, ws = pending.pop(t)
                    lat.append(time.perf_counter() - t0 - arr)
                    done_kinds.append(kind)
                    work += ws
                    t_last = time.perf_counter()
            if now > seconds + drain_s:
                break
            time.sleep(0.0005)
    finally:
        srv.close()
    if backlog_at_end is None:
        backlog_at_end = len(pending)
    elapsed = t_last - t0
    lat = np.array(lat) if lat else np.array([np.nan])
    return {"offered_rate_per_s": rate, "arrival_window_s": seconds, "requests": int(len(arrivals)),
            "completed": int(len(done_kinds)), "unfinished": len(pending),
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 1),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 1),
            "served_req_per_s": round(len(done_kinds) / elapsed, 2) if elapsed > 0 else None,
            "served_world_sim_s_per_s": round(work / elapsed, 1) if elapsed > 0 else None,
            "backlog_at_window_end": int(backlog_at_end),
            "mix": {k: done_kinds.count(k) for k in ("cube", "chain", "box")},
            "requests_shape": "N~U{16..256} candidates, H~U{50..500} x 10 ms, cost+control gradient"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--worlds", type=int, default=4096)
    ap.add_argument("--horizon", type=float, default=0.5)
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--plain-worlds", type=int, default=64)
    ap.add_argument("--cpu-worlds", type=int, default=2048)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="Poisson arrival rate of MPC requests, 1/s")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="arrival window of the serving leg, s")
    ap.add_argument("--no-critical", action="store_true", help="skip the hardest-world-alone leg")
    ap.add_argument("--hardest-only", action="store_true",
                    help="after the counted pass, run only the forward of the world with the most attempts "
                         "(one wavefront; for instruction counters) and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: worlds are independent and this build runs on a single MI355X; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2506_14186_amd import dmx as D
    from paper_2506_14186_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        n = (1 << 30) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 8, "bytes_written": n * 8, "launches": 3}))
        return
    cfg = W.cube_toss(seed=2, n_worlds=args.worlds, horizon=args.horizon)
    model = D.Model(cfg["model"])
    x0 = torch.tensor(cfg["x0"], dtype=torch.float64, device=dev)
    xbar = torch.zeros_like(x0)
    xbar[:, 0:3] = 1.0  # gradient of the summed final positions
    nW, horizon = args.worlds, args.horizon
    fwd_cnt = torch.zeros((nW, len(D.FWD_COUNTERS)), dtype=torch.int64, device=dev)
    adj_cnt = torch.zeros((nW, len(D.ADJ_COUNTERS)), dtype=torch.int64, device=dev)
    tuned = None
    if args.lanes == 0 and not args.no_autotune:
        # team size picked by timing the forward with each compiled one on this batch
        best, times = D.autotune(model, x0, None, 1, horizon)
        tuned = {"lanes_per_world": best, "fwd_ms_by_lanes": {str(k): round(v, 3) for k, v in times.items()}}
    opts = D.default_opts(tape_steps=2048, lanes_per_world=args.lanes)

    # one counted pass (work units), which also allocates the tape reused below
    copts = D.default_opts(tape_steps=2048, lanes_per_world=args.lanes, fwd_counters=fwd_cnt.data_ptr(),
                           adj_counters=adj_cnt.data_ptr())
    r = D.rollout(model, x0, None, 1, horizon, opts=copts, tape=True, counters=True)
    tape = r["tape"]
    g, _ = D.rollout_vjp(tape, xbar)
    torch.cuda.synchronize()
    status = r["status"].cpu().numpy()
    n_acc = r["n_acc"].cpu().numpy()
    fc = dict(zip(D.FWD_COUNTERS, fwd_cnt.sum(0).cpu().numpy().tolist()))
    ac = dict(zip(D.ADJ_COUNTERS, adj_cnt.sum(0).cpu().numpy().tolist()))
    fwd_flops = algorithmic_flops(fc, FWD_FLOPS, model.ncon)
    adj_flops = algorithmic_flops(ac, ADJ_FLOPS, model.ncon)

    n_att = n_acc + r["n_rej"].cpu().numpy()
    hard = int(np.argmax(n_att))

    def alone(reps=3):
        """The hardest world as a batch of one: forward and reverse launch times
        (min over reps) -- the serial chain that bounds the batched launches."""
        x1 = x0[hard:hard + 1].clone()
        o1 = D.default_opts(tape_steps=2048, lanes_per_world=args.lanes or (tuned or {}).get("lanes_per_world", 0))
        r1 = D.rollout(model, x1, None, 1, horizon, opts=o1, tape=True)
        xb1 = xbar[hard:hard + 1].clone()
        D.rollout_vjp(r1["tape"], xb1)
        ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        tf, ta = [], []
        for _ in range(reps):
            ev1[0].record()
            D.rollout(model, x1, None, 1, horizon, opts=o1, reuse=r1["tape"])
            ev1[1].record()
            D.rollout_vjp(r1["tape"], xb1)
            ev1[2].record()
            torch.cuda.synchronize()
            tf.append(ev1[0].elapsed_time(ev1[1])); ta.append(ev1[1].elapsed_time(ev1[2]))
        return min(tf), min(ta)

    if args.hardest_only:
        tf, ta = alone(reps=1)
        print(json.dumps({"hardest_world": hard, "attempts": int(n_att[hard]), "fwd_ms": round(tf, 3),
                          "adj_ms": round(ta, 3)}), flush=True)
        return

    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        rr = D.rollout(model, x0, None, 1, horizon, opts=opts, reuse=tape)
        if ev:
            ev[1].record(stream)
        gg, _ = D.rollout_vjp(rr["tape"], xbar)
        if ev:
            ev[2].record(stream)
        return rr, gg

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    fwd_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    adj_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    value = nW * horizon / (ms_per_step / 1e3)

    dom_name, dom_ms, dom_flops = ("fwd_kernel", fwd_ms, fwd_flops) if fwd_ms >= adj_ms else \
        ("adj_kernel", adj_ms, adj_flops)
    achieved = dom_flops / (dom_ms / 1e3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 4), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_TFLOPS, 6), "traffic": recorded_traffic(dom_name),
                "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)",
                "kernel": dom_name,
                "kernel_ms": round(dom_ms, 3), "flops_per_launch": dom_flops,
                "other_kernel": {"name": "adj_kernel" if dom_name == "fwd_kernel" else "fwd_kernel",
                                 "ms": round(adj_ms if dom_name == "fwd_kernel" else fwd_ms, 3),
                                 "achieved_tflops": round((adj_flops / adj_ms if dom_name == "fwd_kernel"
                                                           else fwd_flops / fwd_ms) / 1e9, 4)}}

    # plain GPU form: the same kernels, one world per launch, on a subset
    plain = None
    if not args.no_plain:
        P = min(args.plain_worlds, nW)
        xs, xbs = x0[:P].contiguous(), xbar[:P].contiguous()
        popts = D.default_opts(tape_steps=2048, lanes_per_world=args.lanes, launch_mode=1)
        rp = D.rollout(model, xs, None, 1, horizon, opts=popts, tape=True)
        D.rollout_vjp(rp["tape"], xbs)
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        rp = D.rollout(model, xs, None, 1, horizon, opts=popts, reuse=rp["tape"])
        D.rollout_vjp(rp["tape"], xbs)
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp0
        plain_value = P * horizon / tp
        plain = {"value": round(plain_value, 2), "unit": "world-sim-s/s", "worlds_timed": P,
                 "ms_for_subset": round(tp * 1e3, 2), "extrapolated_ms_full_batch": round(tp * 1e3 * nW / P, 1),
                 "speedup_batched_over_plain": round(value / plain_value, 2)}

    cpu = None
    if not args.no_cpu:
        from oracle import oracle as O
        S = min(args.cpu_worlds, nW)
        om = O.Model(cfg["model"])
        nthreads = min(16, os.cpu_count() or 1)
        xb = np.zeros((S, 13))
        xb[:, :3] = 1.0
        tc0 = time.perf_counter()
        om.grad_batch(cfg["x0"][:S], None, 1, horizon, xb, n_threads=nthreads)
        tc = time.perf_counter() - tc0
        cpu = {"value": round(S * horizon / tc, 3), "unit": "world-sim-s/s", "cores": nthreads, "kind": "oracle",
               "sample": f"first {S} of the {nW} worlds, full {horizon} s horizon, forward + gradient "
                         f"(forward-mode over the 13 initial-state directions), {tc:.1f} s wall on "
                         f"{nthreads} threads"}

    serving = None
    if not args.no_serve:
        serving = serve_leg(D, W, args.serve_rate, args.serve_seconds)

    critical = None
    if not args.no_critical:
        tf, ta = alone()
        critical = {"world": hard, "attempts": int(n_att[hard]), "accepted": int(n_acc[hard]),
                    "attempts_mean": round(float(n_att.mean()), 1),
                    "alone_fwd_ms": round(tf, 3), "alone_adj_ms": round(ta, 3),
                    "alone_us_per_attempt": round(tf * 1e3 / float(n_att[hard]), 2),
                    "batch_fwd_ms": round(fwd_ms, 3), "batch_adj_ms": round(adj_ms, 3)}

    out = {
        "metric": "sim-seconds/s fwd+adjoint at rtol 1e-6 vs plain GPU form; p99 request latency",
        "value": round(value, 2),
        "unit": "world-sim-s/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"cube_toss: {nW} free cubes x 8 corner contacts, {horizon} s, t_c 1 ms, "
                               f"rtol 1e-6 atol 1e-8, fwd + adjoint of summed final position",
                   "worlds": nW, "horizon_s": horizon,
                   "lanes_per_world": args.lanes or (tuned["lanes_per_world"] if tuned else "default"),
                   "autotune": tuned,
                   "parallelism": "1 GPU, worlds batched in one launch"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "plain_gpu": plain,
        "serving": serving,
        "critical_path": critical,
        "work": {"fwd": fc, "adj": ac, "accepted_steps_mean": float(n_acc.mean()),
                 "accepted_steps_max": int(n_acc.max()), "failed_worlds": int((status != 0).sum()),
                 "fwd_ms": round(fwd_ms, 3), "adj_ms": round(adj_ms, 3)},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
