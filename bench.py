#!/usr/bin/env python
"""Benchmark of the contact-manifold hot path on one MI355X.

A step is one pass of the whole path over the batch: broad phase, vertex-SDF
and edge-SDF narrow phase, mollification and per-piece blending (the group
records), the adjoint w.r.t. both 6-DoF poses (gradient) and the
Hessian-vector product along a unit direction, as one cm_contacts_step call
(one forward sweep in dual numbers that keeps the adjoint tape, one adjoint)
on the 16384-pair workload with log-uniform piece counts [1, 32] and hull
sizes [8, 512] (synthetic, seeded).  `value` is whole-batch pair-queries per
second with the inputs resident in device memory.  The same outputs from the
three separate calls (cm_contacts_fwd + cm_contacts_bwd + cm_hvp) and the
forward + gradient step without H v are timed beside it.

Beside it the JSON line carries:
  roofline      the dominant narrow-phase kernel's algorithmic VALU lane-ops
                per second (HIP events on the launch stream) against the chip's
                FP32 VALU issue rate (256 CU x 4 SIMD x 16 lanes x 2.4 GHz);
  cpu_baseline  the FP64 oracle (forward + hyper-dual gradient and HVP) on a
                bounded sample of the same workload, on the host's cores;
  plain_launch  the same kernels launched one pair-query at a time;
  parity        sampled GPU-vs-oracle errors at the benchmark's launch shape.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9  # FP32 VALU lane-ops/s (non-packed issue rate)
K_TRACE = 3
# Algorithmic VALU lane-ops per (point, opposing plane) for an SDF evaluation
# returning the value (7: 3 FMA dot, max, shift, exp, add), + gradient (10:
# + 3 FMA), + Hessian (16: + 6 FMA); in dual numbers 12, 18 and 30.  A
# surviving vertex is one evaluation, a surviving edge 2K trace evaluations
# plus one at the edge point.  Per (vertex, plane) and (edge, plane):
OPS = {
    "forward": (10, 2 * K_TRACE * 7 + 10),             # value + gradient at the contact
    "forward_tape": (16, 2 * K_TRACE * 10 + 16),       # + trace gradients and Hessian (before an adjoint)
    "forward_tape_dual": (30, 2 * K_TRACE * 18 + 30),  # the same in dual numbers (before H v)
}


TRAFFIC_PROFILE = os.path.join(HERE, "profiles", "k_narrow_dual_tape_c2_16384pairs_hbm_traffic.txt")
DOMINANT = "k_narrow<df, false, true>"


def kernel_source_hash():
    import glob
    import hashlib
    h = hashlib.sha256()
    src = os.path.join(HERE, "paper_2604_17538_amd", "csrc")
    for p in sorted(glob.glob(os.path.join(src, "*.hip")) + glob.glob(os.path.join(src, "*.h"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(config="c2", pairs=None):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a 1 GiB copy), or None when the
    kernel sources changed since the counters were taken or the workload is not
    the one they were taken on (C2 at its full 16384 pair-queries)."""
    if config != "c2" or pairs not in (None, 16384):
        return None
    try:
        with open(TRAFFIC_PROFILE) as f:
            lines = f.read().splitlines()
    except OSError:
        return None
    tag = "kernel sources sha256[:16] (csrc/*.hip, *.h): "
    h = [l[len(tag):].strip() for l in lines if l.startswith(tag)]
    if not h or h[0] != kernel_source_hash():
        return None
    for l in lines:
        if l.startswith(DOMINANT):
            v = l[len(DOMINANT):].split()
            return (float(v[2]) + float(v[3])) * 1e9
    return None


def log(msg):
    print("[bench %.1fs] %s" % (time.time() - T0, msg), file=sys.stderr, flush=True)


T0 = time.time()


def build_workload(cfg, pairs):
    from paper_2604_17538_amd import workloads as W
    if cfg == "c0":
        return W.config0()
    if cfg == "c1":
        return W.config1(n_envs=pairs or 4096)
    if cfg == "c2":
        return W.config2(n_pairs=pairs or 16384)
    if cfg == "c4":
        return W.config4(n_envs=pairs or 65536, library=2048)
    raise ValueError(cfg)


# device-memory budget of the context per workload (a quarter of it holds the
# adjoint tape; tiles past it are recomputed by the adjoint)
BUDGET_GB = {"c0": 32, "c1": 32, "c2": 32, "c4": 256}


def cpu_baseline(w, sample, threads, want_grad=True):
    """Oracle (FP64, OpenMP over pair-queries) on the first `sample` queries."""
    import oracle as O
    prm = O.default_params(w.L_ref)
    sel = np.arange(min(sample, w.n))
    objs = [None] * len(w.objects)
    for i in sel:
        for j in (w.qa[i], w.qb[i]):
            if objs[j] is None:
                objs[j] = O.from_workload_object(w.objects[j])
                objs[j].build_grid(prm)
    t = time.time()
    g, goff = O.contacts(prm, objs, w.qa[sel], w.qb[sel], w.poses[sel], threads=threads)
    from paper_2604_17538_amd import workloads as W
    cot = W.cotangents(w.cot_seed or 1, goff[-1])
    d = W.directions(w.cot_seed or 1, len(sel))
    grad, hv = O.grad_hvp(prm, objs, w.qa[sel], w.qb[sel], w.poses[sel], cot, d, threads=threads)
    dt = time.time() - t
    return dict(sel=sel, groups=g, goff=goff, grad=grad, hv=hv, cot=cot, dir=d, seconds=dt)


def serving_leg(api, W, rates, seconds):
    """Poisson request streams over a library of 2048 resident objects (pieces
    as in the differentiation workload): each request U{1..64} pairs, 70 %
    forward, 30 % forward + gradient, admitted under a 32 GB budget.  Requests
    are submitted at their arrival times; latency is the library's own record
    from cm_submit to results written."""
    lib = W.library_objects(2048)
    ctx = api.Context(0, L_ref=0.1, budget_bytes=32 << 30)
    hs = ctx.build_objects(lib)
    srv = api.Server(ctx)
    out = []
    for k, rate in enumerate(rates):
        tr = W.serving_trace(lib, rate_hz=rate, duration_s=seconds, seed=W.SEED_BASE + 3 + k)
        rng = np.random.default_rng(11 + k)
        reqs = []
        for r in range(len(tr.arrival_s)):
            a, b = hs[tr.pair_a[r]], hs[tr.pair_b[r]]
            cot = None
            if tr.want_grad[r]:
                G = sum(srv._pieces(int(x)) + srv._pieces(int(y)) for x, y in zip(a, b))
                cot = rng.standard_normal((G, 12))
            reqs.append((a, b, tr.poses[r], cot))
        srv.latencies()  # drop earlier records
        b0 = srv.stats()["batches"]
        tickets = []
        t0 = time.perf_counter()
        late = 0.0
        for r, (a, b, ps, cot) in enumerate(reqs):
            while True:
                now = time.perf_counter() - t0
                if now >= tr.arrival_s[r]:
                    break
                if tr.arrival_s[r] - now > 2e-4:
                    time.sleep(1e-4)
            late = max(late, now - tr.arrival_s[r])
            tickets.append(srv.submit(a, b, ps, cot))
        for t in tickets:
            t.wait(120000)
        wall = time.perf_counter() - t0
        lat = srv.latencies() * 1e3
        pairs = int(sum(len(x[0]) for x in reqs))
        b1 = srv.stats()["batches"]
        out.append({"rate_req_s": rate, "requests": len(reqs), "pairs": pairs,
                    "throughput_req_s": round(len(reqs) / wall, 1), "pair_queries_s": round(pairs / wall, 1),
                    "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
                    "max_submit_lag_ms": round(late * 1e3, 3), "batches": b1 - b0})
    return out


def sweep_leg(reps=10):
    """Broad + narrow phase against narrow phase only (the design of Sec. V.4):
    one pair of the 8-piece workload, 1024 translations of B along x linearly
    spaced over [1, 2] times the x-extent of A's bounding box (identity
    rotations), forward records of the batch timed with the broad phase on and
    off for d_max at 0, 0.25, 0.5, 1 and 2 times its default."""
    import torch
    from paper_2604_17538_amd import api, workloads as W
    w = W.config1(n_envs=1)
    objs = [w.objects[0], w.objects[1]]
    ext = float(np.ptp(objs[0].points[:, 0]))
    n = 1024
    poses = np.zeros((n, 14))
    poses[:, 0] = 1.0
    poses[:, 7] = 1.0
    poses[:, 11] = np.linspace(1.0, 2.0, n) * ext
    poses = W._f32(poses)
    d0 = api.default_params(w.L_ref).d_max
    stream = torch.cuda.current_stream()
    rows = []
    for f in (0.0, 0.25, 0.5, 1.0, 2.0):
        for bp in (1, 0):
            ctx = api.Context(0, L_ref=w.L_ref, d_max=d0 * f, broad_phase=bp)
            hs = ctx.build_objects(objs)
            plan = ctx.plan(np.repeat(hs[:1], n), np.repeat(hs[1:], n))
            qd = plan.device_queries(poses)
            out = plan.forward(qd, stream=stream)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                plan.forward(qd, out=out, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            st = plan.stats()
            rows.append({"d_max_factor": f, "broad_phase": bp, "ms": round(a.elapsed_time(b) / reps, 4),
                         "surviving_contacts": st["surv_verts"] + st["surv_edges"],
                         "contacts": st["verts"] + st["edges"]})
            log("sweep %s" % rows[-1])
            del plan, ctx
    return {"pair_queries": n, "x_extent_A": round(ext, 5), "translation_factors": [1.0, 2.0], "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2", choices=["c0", "c1", "c2", "c4"])
    ap.add_argument("--pairs", type=int, default=None, help="batch size override (default: the config's)")
    ap.add_argument("--budget-gb", type=float, default=None, help="device-memory budget (default per workload)")
    ap.add_argument("--no-prune", action="store_true", help="evaluate every piece (no piece pruning)")
    ap.add_argument("--cpu-sample", type=int, default=16)
    ap.add_argument("--plain-sample", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-separate", action="store_true", help="skip timing the three separate calls")
    ap.add_argument("--no-tight", action="store_true", help="skip the step with the tighter edge bound")
    ap.add_argument("--launch-shape", default=None,
                    help="F,D: fixed persistent workgroups per CU for the float and dual sweeps (no autotuning)")
    ap.add_argument("--tune-sample", type=int, default=16384,
                    help="autotune on a plan of the first N pair-queries when the batch is larger")
    ap.add_argument("--sweep", action="store_true",
                    help="only the broad-phase sweep (broad + narrow vs narrow only over d_max); prints its own JSON line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device copy of 1 GiB three times (scale of the HBM traffic counters)")
    ap.add_argument("--serve-rates", default="2000,5000", help="Poisson request rates (req/s) for the serving leg")
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: pair-queries are independent and the path has no "
              "cross-GPU step; run with --gpus 1 (several GPUs would each run their own share of the "
              "pair-queries, with no communication)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4, "dispatches": 3}))
        return
    from paper_2604_17538_amd import api, workloads as W
    if args.sweep:
        print(json.dumps({"sweep": sweep_leg()}), flush=True)
        return

    w = build_workload(args.config, args.pairs)
    log("workload %s: %d pair-queries, %d objects" % (args.config, w.n, len(w.objects)))
    budget_gb = args.budget_gb or BUDGET_GB[args.config]
    ctx = api.Context(0, L_ref=w.L_ref, budget_bytes=int(budget_gb * (1 << 30)), prune_pieces=0 if args.no_prune else 1)
    hs = ctx.build_objects(w.objects)
    torch.cuda.synchronize()
    log("objects resident")
    plan = ctx.plan(hs[w.qa], hs[w.qb])
    qd = plan.device_queries(w.poses)
    cot = W.cotangents(w.cot_seed or 1, plan.G)
    direc = W.directions(w.cot_seed or 1, w.n)
    cot_d = torch.tensor(cot.T.astype(np.float32)).contiguous().cuda()
    dir_d = torch.tensor(direc.astype(np.float32)).cuda()
    out = torch.empty((12, plan.G), dtype=torch.float32, device="cuda")
    grad = torch.empty((w.n, 12), dtype=torch.float32, device="cuda")
    grad2 = torch.empty_like(grad)
    hv = torch.empty_like(grad)
    stream = torch.cuda.current_stream()

    def step():
        plan.step(qd, cot_d, dir_d, out=out, grad=grad, hv=hv, stream=stream)

    def separate():
        plan.forward(qd, out=out, stream=stream)
        plan.backward(qd, cot_d, grad=grad2, stream=stream)
        plan.hvp(qd, cot_d, dir_d, hv=hv, grad=grad2, stream=stream)

    def fwd_grad():
        plan.step(qd, cot_d, out=out, grad=grad2, stream=stream)

    def timed(fn, reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        torch.cuda.synchronize()
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    # launch shapes picked by the autotuner (persistent workgroups per CU), one
    # for the sweeps in dual numbers (this step) and one for the float sweeps
    if args.launch_shape:
        shape_f, shape = (int(v) for v in args.launch_shape.split(","))
        plan.launch_shape = (shape_f, shape)
        tuned_on = 0
    elif w.n <= args.tune_sample:
        shape = plan.autotune(qd, cot_d, grad, dir_d, hv, stream)
        shape_f = plan.autotune(qd, cot_d, grad, stream=stream)
        tuned_on = w.n
    else:
        # a large batch: tune on a plan of its first pair-queries, apply to the whole
        ns = args.tune_sample
        tp = ctx.plan(hs[w.qa[:ns]], hs[w.qb[:ns]])
        tq = tp.device_queries(w.poses[:ns])
        tc = cot_d[:, : tp.G].contiguous()
        tg = torch.empty((ns, 12), dtype=torch.float32, device="cuda")
        shape = tp.autotune(tq, tc, tg, dir_d[:ns].contiguous(), torch.empty_like(tg), stream)
        shape_f = tp.autotune(tq, tc, tg, stream=stream)
        plan.launch_shape = (shape_f, shape)
        del tp, tq, tc, tg
        tuned_on = ns
    how = ("autotuned on %d pair-queries" % tuned_on) if tuned_on else "set by --launch-shape"
    log("launch shape (%s): %d workgroups per CU (dual sweeps), %d (float sweeps)" % (how, shape, shape_f))
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.time()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.time() - t_wall
    ms = e0.elapsed_time(e1) / args.steps
    log("timed %d steps: %.2f ms/step (wall %.2f s)" % (args.steps, ms, wall))

    # the same outputs by the separate calls, and the forward + gradient step
    sep_ms = None if args.no_separate else timed(separate, 2)
    fg_ms = timed(fwd_grad, 1 if w.n > args.tune_sample else 2)
    fw_ms = timed(lambda: plan.forward(qd, out=out, stream=stream), 1 if w.n > args.tune_sample else 2)
    log("separate calls %s ms, forward + gradient step %.2f ms, forward %.2f ms" % (sep_ms, fg_ms, fw_ms))
    # the step replayed from a HIP graph of its launches
    graph = plan.graph(qd, cot_d, grad, dir_d, hv, out)
    graph_ms = timed(lambda: graph.launch(stream), max(args.steps, 1 if w.n > args.tune_sample else 2))
    del graph
    log("graph replay %.2f ms" % graph_ms)

    # the same step with the tighter edge bound of the broad phase (outputs are
    # unchanged, only the candidate lists shrink), in a context of its own
    tight = None
    if not args.no_tight and args.config != "c4":  # (c4: a second plan would double ~80 GB of scratch)
        ctx_t = api.Context(0, L_ref=w.L_ref, budget_bytes=int(budget_gb * (1 << 30)), edge_bound=1)
        hs_t = ctx_t.build_objects(w.objects)
        plan_t = ctx_t.plan(hs_t[w.qa], hs_t[w.qb])
        plan_t.launch_shape = plan.launch_shape
        qd_t = plan_t.device_queries(w.poses)
        out_t, grad_t, hv_t = torch.empty_like(out), torch.empty_like(grad), torch.empty_like(hv)
        t_ms = timed(lambda: plan_t.step(qd_t, cot_d, dir_d, out=out_t, grad=grad_t, hv=hv_t, stream=stream),
                     max(args.steps, 1 if w.n > args.tune_sample else 2))
        st_t = plan_t.stats()
        tight = {"ms_per_step": round(t_ms, 3), "value": round(w.n / (t_ms * 1e-3), 1),
                 "surviving_contacts": st_t["surv_verts"] + st_t["surv_edges"],
                 "note": "edge bound max(max(lb1, lb2) - l, (lb1 + lb2 - l) / 2) instead of min(lb1, lb2) - l"}
        log("tight edge bound %s" % tight)
        del plan_t, qd_t, ctx_t, out_t, grad_t, hv_t

    # per-kernel timing of the step (events on the launch stream), untimed region
    plan.set_timing(True)
    step()
    torch.cuda.synchronize()
    tk = plan.timing()
    plan.set_timing(False)
    work_v, work_e = plan.work()
    split = {k: round(v, 3) for k, v in tk.items() if v >= 0}
    st = plan.stats()
    dom_ms = tk["narrow_tan"]  # the dual forward sweep keeping the tape
    ov, oe = OPS["forward_tape_dual"]
    alg_ops = st["vertex_pairs"] * ov + st["edge_pairs"] * oe
    achieved = alg_ops / (dom_ms * 1e-3)
    # the same per-pair costs over the evaluations the kernel performed (after
    # piece pruning, all 64 lanes of every tile, plus the pruning bounds)
    rho_v = work_v / max(st["vertex_pairs"], 1)
    rho_e = work_e / max(st["edge_pairs"] * (2 * K_TRACE + 1), 1)
    perf_ops = rho_v * st["vertex_pairs"] * ov + rho_e * st["edge_pairs"] * oe
    perf_achieved = perf_ops / (dom_ms * 1e-3)
    roofline = {"bound": "alu", "kernel": "k_narrow<df, forward, tape>", "achieved": round(achieved / 1e12, 3),
                "peak": round(PEAK_LANE_OPS / 1e12, 3), "unit": "T lane-op/s (FP32 VALU)",
                "frac": round(achieved / PEAK_LANE_OPS, 4), "traffic": measured_traffic(args.config, args.pairs),
                "kernel_ms": round(dom_ms, 3), "alg_ops_per_launch": int(alg_ops),
                "algorithmic_point_plane": int(st["pairs"]), "performed_point_plane": int(work_v + work_e),
                "performed_achieved": round(perf_achieved / 1e12, 3),
                "performed_frac": round(perf_achieved / PEAK_LANE_OPS, 4)}
    log("roofline %s" % roofline)

    # the forward pass alone (records only): its narrow-phase kernel against the same peak
    plan.set_timing(True)
    plan.forward(qd, out=out, stream=stream)
    torch.cuda.synchronize()
    fwd_k = plan.timing()["narrow_fwd"]
    plan.set_timing(False)
    fv, fe = OPS["forward"]
    f_ops = st["vertex_pairs"] * fv + st["edge_pairs"] * fe
    forward_roofline = {"bound": "alu", "kernel": "k_narrow<float, forward>", "kernel_ms": round(fwd_k, 3),
                        "achieved": round(f_ops / (fwd_k * 1e-3) / 1e12, 3), "unit": "T lane-op/s (FP32 VALU)",
                        "frac": round(f_ops / (fwd_k * 1e-3) / PEAK_LANE_OPS, 4), "alg_ops_per_launch": int(f_ops)}
    log("forward roofline %s" % forward_roofline)

    # plain per-pair launch: same kernels, one pair-query per launch
    plain = None
    if not args.no_plain:
        ns = min(args.plain_sample, w.n)
        plans = []
        for i in range(ns):
            p1 = ctx.plan(hs[w.qa[i:i + 1]], hs[w.qb[i:i + 1]])
            q1 = p1.device_queries(w.poses[i:i + 1])
            g0, g1 = plan.group_off[i], plan.group_off[i + 1]
            c1 = cot_d[:, g0:g1].contiguous()
            o1 = torch.empty((12, p1.G), dtype=torch.float32, device="cuda")
            gr1 = torch.empty((1, 12), dtype=torch.float32, device="cuda")
            plans.append((p1, q1, c1, dir_d[i:i + 1].contiguous(), o1, gr1, torch.empty_like(gr1),
                          torch.empty_like(gr1)))

        def plain_pass():
            for p1, q1, c1, d1, o1, gr1, gr2, hv1 in plans:
                p1.step(q1, c1, d1, out=o1, grad=gr1, hv=hv1, stream=stream)

        plain_pass()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        plain_pass()
        b.record(stream)
        torch.cuda.synchronize()
        pms = a.elapsed_time(b)
        batched_sample_rate = None
        plain = {"sample": ns, "ms": round(pms, 3), "value": round(ns / (pms * 1e-3), 1), "unit": "pair-queries/s",
                 "note": "first %d pair-queries, one cm_contacts_step (records + gradient + H v) per query, same kernels" % ns}
        log("plain launch %s" % plain)

    # parity on sampled outputs of the step against the oracle, plus the CPU baseline timing
    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        step()
        torch.cuda.synchronize()
        threads = min(os.cpu_count() or 1, 16)
        res = cpu_baseline(w, args.cpu_sample, threads)
        ns = len(res["sel"])
        cpu = {"value": round(ns / res["seconds"], 4), "unit": "pair-queries/s", "cores": threads, "kind": "oracle",
               "sample": "first %d pair-queries of the workload, FP64 forward + hyper-dual gradient and HVP, "
                         "OpenMP over queries (%.1f s)" % (ns, res["seconds"])}
        g_gpu = out.cpu().numpy().T.astype(np.float64)[: plan.group_off[ns]]
        r = np.array([o.radius() for o in w.objects])
        Ls = np.repeat(r[w.qa[:ns]] + r[w.qb[:ns]], np.diff(plan.group_off[: ns + 1]))
        pos = np.abs(g_gpu[:, [0, 1, 2, 6, 7, 8, 9]] - res["groups"][:, [0, 1, 2, 6, 7, 8, 9]]).max(1) / Ls
        gg = grad.cpu().numpy()[:ns].astype(np.float64)
        hh = hv.cpu().numpy()[:ns].astype(np.float64)
        # the oracle used the same cotangents and directions for these queries
        gerr = np.linalg.norm(gg - res["grad"], axis=1) / np.maximum(np.linalg.norm(res["grad"], axis=1), 1e-30)
        herr = np.linalg.norm(hh - res["hv"], axis=1) / np.maximum(np.linalg.norm(res["hv"], axis=1), 1e-30)
        parity = {"queries": ns, "max_pos_err_over_Ls": float(pos.max()), "max_grad_rel_err": float(gerr.max()),
                  "max_hvp_rel_err": float(herr.max())}
        log("cpu baseline %s parity %s" % (cpu, parity))

    serving = None
    if not args.no_serving:
        serving = serving_leg(api, W, [float(r) for r in args.serve_rates.split(",")], args.serve_seconds)
        log("serving %s" % serving)

    value = w.n / (ms * 1e-3)
    line = {
        "metric": "pair-queries/s fwd+grad at 1e-5 err vs plain launch; p50/p99 request latency",
        "value": round(value, 1),
        "unit": "pair-queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s: %d pair-queries, forward + gradient (both poses) + HVP per step" % (args.config, w.n),
                   "pair_queries": w.n, "groups": plan.G, "contacts": plan.C, "step": "cm_contacts_step",
                   "budget_gb": budget_gb},
        "split_ms": split,
        "separate_calls_ms_per_step": round(sep_ms, 3) if sep_ms is not None else None,
        "graph_replay_ms_per_step": round(graph_ms, 3),
        "launch_shape": {"workgroups_per_cu": shape, "workgroups_per_cu_float": shape_f,
                         "tile": "one wave of 64 contacts", "tuned_on_pair_queries": tuned_on},
        "forward_gradient_step_ms": round(fg_ms, 3),
        "forward_gradient_value": round(w.n / (fg_ms * 1e-3), 1),
        "forward_ms": round(fw_ms, 3),
        "forward_roofline": forward_roofline,
        "tight_edge_bound": tight,
        "forward_value": round(w.n / (fw_ms * 1e-3), 1),
        "work": st,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "plain_launch": plain,
        "parity": parity,
        "serving": serving,
    }
    if plain:
        line["vs_plain_launch"] = round(value / plain["value"], 2)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
