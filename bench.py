#!/usr/bin/env python
"""Benchmark of the contact-manifold hot path on one MI355X.

A step is one pass of the whole path over the batch: broad phase, vertex-SDF
and edge-SDF narrow phase, mollification and per-piece blending (the group
records), the adjoint w.r.t. both 6-DoF poses (gradient) and the
Hessian-vector product along a unit direction, as one cm_contacts_step call
(one forward sweep in dual numbers that keeps the adjoint tape, one adjoint).
The default workload is the large batched one: 65536 pair-queries of
32-piece objects (hulls of log-uniform [64, 1024] ellipsoid points, drawn
from a library of 2048 objects), synthetic and seeded.  `value` is
whole-batch pair-queries per second with the inputs resident in device
memory.  The forward + gradient step without H v, the forward pass alone and
the step replayed from its HIP graph are timed beside it, and the same step on
the 16384-pair differentiation workload as a secondary figure.

Beside it the JSON line carries:
  roofline      the dominant narrow-phase kernel's algorithmic VALU lane-ops
                per second (HIP events on the launch stream) against the chip's
                FP32 VALU issue rate (256 CU x 4 SIMD x 16 lanes x 2.4 GHz), and
                the same per-pair costs over the work the kernel performed;
  cpu_baseline  the FP64 oracle on a bounded sample of the same workload, on the
                host's cores (run in a child process while the GPU legs run);
  plain_launch  the same kernels launched one pair-query at a time;
  parity        the step's outputs at sampled queries against stored FP64 oracle
                values (large workload) or the oracle run here (others);
  serving       Poisson request streams through cm_submit / cm_poll.
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


DOMINANT = "k_narrow<df, false, true, 0>"  # the forward sweep in dual numbers keeping the tape (plane SDFs)
HERE_PROFILES = os.path.join(HERE, "profiles")
KERNEL_FILES = ("common.h", "devmath.h", "kernels.h", "wave.h")  # headers the kernels include


def kernel_source_hash():
    """sha256[:16] over the kernel sources (csrc/*.hip and the headers they include)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    src = os.path.join(HERE, "paper_2604_17538_amd", "csrc")
    files = sorted(glob.glob(os.path.join(src, "*.hip")) + [os.path.join(src, f) for f in KERNEL_FILES])
    for p in files:
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(config, pairs):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary of this workload (FETCH_SIZE and WRITE_SIZE scaled by a 1 GiB
    copy), or None when there is none or the kernel sources changed since the
    counters were taken."""
    path = os.path.join(HERE_PROFILES, "k_narrow_dual_tape_%s_%dpairs_hbm_traffic.txt" % (config, pairs))
    try:
        with open(path) as f:
            lines = f.read().splitlines()
    except OSError:
        return None
    tag = "kernel sources sha256[:16]"
    h = [l.rsplit(":", 1)[1].strip() for l in lines if l.startswith(tag)]
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
# the FP64 oracle's sample per workload: (queries, with gradient and H v);
# the 32-piece workload takes minutes of hyper-dual arithmetic per query, so
# only its forward records are timed there
CPU_SAMPLE = {"c0": (64, True), "c1": (16, True), "c2": (16, True), "c4": (8, False)}


def cpu_child(spec):
    """Child process: the oracle (FP64, OpenMP over pair-queries) on the first
    queries of the workload; prints one JSON line with the timing and results."""
    import oracle as O
    from paper_2604_17538_amd import workloads as W
    w = build_workload(spec["config"], spec["pairs"])
    prm = O.default_params(w.L_ref)
    sel = np.arange(min(spec["sample"], w.n))
    objs = [None] * len(w.objects)
    t0 = time.time()
    for i in sel:
        for j in (w.qa[i], w.qb[i]):
            if objs[j] is None:
                objs[j] = O.from_workload_object(w.objects[j])
                objs[j].build_grid(prm)
    t_obj = time.time() - t0
    t = time.time()
    g, goff = O.contacts(prm, objs, w.qa[sel], w.qb[sel], w.poses[sel], threads=spec["threads"])
    res = dict(n=len(sel), objects_s=t_obj, groups=g.tolist(), goff=goff.tolist(),
               radii=[objs[j].radius() if objs[j] is not None else 0.0 for j in range(len(objs))])
    if spec["grad"]:
        cot = np.asarray(spec["cot"], np.float64).reshape(-1, 12)[: goff[-1]]
        d = np.asarray(spec["dir"], np.float64).reshape(-1, 12)[: len(sel)]
        grad, hv = O.grad_hvp(prm, objs, w.qa[sel], w.qb[sel], w.poses[sel], cot, d, threads=spec["threads"])
        res.update(grad=grad.tolist(), hv=hv.tolist())
    res["seconds"] = time.time() - t
    print(json.dumps(res), flush=True)


def start_cpu_child(config, pairs, cot, direc, threads):
    """Starts the oracle leg in a child process (it runs while the GPU legs
    run; its own timing covers only the oracle's evaluation)."""
    import subprocess
    sample, grad = CPU_SAMPLE[config]
    spec = dict(config=config, pairs=pairs, sample=sample, grad=grad, threads=threads,
                cot=cot.tolist() if grad else None,
                dir=direc[:sample].tolist() if grad else None)
    import tempfile
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    fd, path = tempfile.mkstemp(suffix=".json", prefix="cm_cpu_child_")
    with os.fdopen(fd, "w") as f:
        json.dump(spec, f)
    p = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-child", path],
                         stdout=subprocess.PIPE, text=True, env=env, cwd=HERE)
    return p, spec


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


def curve_study_leg(n_pairs=1024, reps=5):
    """Serialization study (Sec. IV-C.3): the vertices and edges of each piece
    ordered along no curve, a Morton (Z-order) curve or a Hilbert curve.  For the
    8-piece workload: the fraction of mixed chunks (consecutive contacts of one
    piece and kind, 32 or 64 at a time, that the broad phase partly accepts and
    partly filters: the divergence the paper's ordering targets), and the broad
    and narrow phase times of the forward pass (events on the launch stream)."""
    import torch
    from paper_2604_17538_amd import api, workloads as W
    w = W.config1(n_envs=n_pairs)
    stream = torch.cuda.current_stream()
    rows = []
    for curve, name in ((0, "none"), (1, "morton"), (2, "hilbert")):
        ctx = api.Context(0, L_ref=w.L_ref, curve=curve)
        hs = ctx.build_objects(w.objects)
        plan = ctx.plan(hs[w.qa], hs[w.qb])
        qd = plan.device_queries(w.poses)
        out, dbg = plan.forward(qd, debug=True, stream=stream)
        torch.cuda.synchronize()
        mask = dbg[0].cpu().numpy() > 0.5
        # segment boundaries: per query, A's pieces then B's; per piece vertices then edges
        ex = {}
        seg_len = []
        for a, b in zip(w.qa, w.qb):
            for j in (a, b):
                if j not in ex:
                    e = ctx.object_export(hs[j])
                    ex[j] = np.stack([np.diff(e["vert_off"]), np.diff(e["edge_off"])], 1).ravel()
                seg_len.append(ex[j])
        seg_len = np.concatenate(seg_len)
        seg = np.repeat(np.arange(len(seg_len)), seg_len)
        pos = np.arange(len(seg)) - np.repeat(np.cumsum(seg_len) - seg_len, seg_len)
        res = {"curve": name}
        for width in (32, 64):
            key = seg.astype(np.int64) * 1_000_000 + pos // width
            _, inv = np.unique(key, return_inverse=True)
            acc = np.bincount(inv, weights=mask.astype(np.float64))
            cnt = np.bincount(inv)
            mixed = (acc > 0) & (acc < cnt)
            res["mixed_chunks_%d" % width] = round(float(mixed.mean()), 4)
        plan.set_timing(True)
        tb, tn = [], []
        for _ in range(reps):
            plan.forward(qd, out=out, stream=stream)
            torch.cuda.synchronize()
            t = plan.timing()
            tb.append(t["broad"])
            tn.append(t["narrow_fwd"])
        res.update(broad_ms=round(float(np.median(tb)), 4), narrow_ms=round(float(np.median(tn)), 4),
                   survivors=round(float(mask.mean()), 4))
        rows.append(res)
        log("curve study %s" % res)
        del plan, ctx, dbg
        torch.cuda.empty_cache()
    return {"workload": "c1: %d pair-queries of 8-piece objects, forward" % n_pairs, "rows": rows}


def spline_leg(n_pairs=2048, reps=5):
    """The spline SDF representation (Sec. III-B) on the 8-piece workload:
    every object's SDF a cubic spline over a 32^3-cell box (with a fitted normal
    spline), fitted on the device at registration.  Times the forward records
    and the step (records + gradient + H v) of the batch, beside the plane
    representation on the same batch; a spline evaluation gathers 64
    coefficients of 16 bytes."""
    import torch
    from paper_2604_17538_amd import api, workloads as W
    w = W.config1(n_envs=n_pairs)
    stream = torch.cuda.current_stream()
    out = {"workload": "c1: %d pair-queries of 8-piece objects" % n_pairs}
    for name, kw in (("spline", dict(sdf_kind=1, grid_margin_rel=0.0)), ("planes", {})):
        ctx = api.Context(0, L_ref=w.L_ref, **kw)
        torch.cuda.synchronize()
        t0 = time.time()
        hs = ctx.build_objects(w.objects)
        torch.cuda.synchronize()
        t_build = time.time() - t0
        plan = ctx.plan(hs[w.qa], hs[w.qb])
        qd = plan.device_queries(w.poses)
        cot = torch.tensor(np.ascontiguousarray(W.cotangents(5, plan.G).T, np.float32)).cuda()
        direc = torch.tensor(W.directions(5, w.n).astype(np.float32)).cuda()
        o = plan.forward(qd, stream=stream)
        res = {}
        for what, fn in (("forward", lambda: plan.forward(qd, out=o, stream=stream)),
                         ("step", lambda: plan.step(qd, cot, direc, stream=stream))):
            fn()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                fn()
            b.record(stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            res[what + "_ms"] = round(ms, 3)
            res[what + "_value"] = round(w.n / (ms * 1e-3), 1)
        plan.set_timing(True)
        plan.forward(qd, out=o, stream=stream)
        torch.cuda.synchronize()
        k_ms = plan.timing()["narrow_fwd"]
        wv, we = plan.work()
        plan.set_timing(False)
        st = plan.stats()
        res.update(build_s=round(t_build, 2), narrow_fwd_ms=round(k_ms, 3),
                   surviving_contacts=st["surv_verts"] + st["surv_edges"])
        if name == "spline":
            evals = (wv + we) / 64
            res.update(evaluations=int(evals), evaluations_per_s=round(evals / (k_ms * 1e-3), 1),
                       gather_GBps=round(evals * 64 * 16 / (k_ms * 1e-3) / 1e9, 1))
        out[name] = res
        log("spline leg %s %s" % (name, res))
        del plan, ctx
        torch.cuda.empty_cache()
    return out


def prims_leg(n_pairs=4096, reps=5):
    """The primitive representation (Sec. III-A: PSQs and XPSQs folded by
    union / subtraction / intersection) on pairs of cup / tube / dome /
    rounded-box objects: forward records and the step (records + gradient +
    H v), evaluations per second of the primitive SDF (every contact survives:
    primitives carry no broad-phase bound)."""
    import torch
    from paper_2604_17538_amd import api, workloads as W
    w = W.config_prims(n_pairs=n_pairs)
    stream = torch.cuda.current_stream()
    ctx = api.Context(0, L_ref=w.L_ref, sdf_kind=2)
    hs = ctx.build_objects(w.objects)
    plan = ctx.plan(hs[w.qa], hs[w.qb])
    qd = plan.device_queries(w.poses)
    cot = torch.tensor(np.ascontiguousarray(W.cotangents(5, plan.G).T, np.float32)).cuda()
    direc = torch.tensor(W.directions(5, w.n).astype(np.float32)).cuda()
    o = plan.forward(qd, stream=stream)
    res = {"workload": "prims: %d pair-queries of primitive objects (cup, tube, dome, rounded box)" % w.n,
           "contacts": plan.C, "groups": plan.G}
    for what, fn in (("forward", lambda: plan.forward(qd, out=o, stream=stream)),
                     ("step", lambda: plan.step(qd, cot, direc, stream=stream))):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        res[what + "_ms"] = round(ms, 3)
        res[what + "_value"] = round(w.n / (ms * 1e-3), 1)
    plan.set_timing(True)
    plan.forward(qd, out=o, stream=stream)
    torch.cuda.synchronize()
    k_ms = plan.timing()["narrow_fwd"]
    plan.set_timing(False)
    st = plan.stats()
    # evaluations of the object SDF by the forward sweep: a vertex once, an edge 2K + 1 times
    K2 = 2 * ctx.params.st_iters + 1
    evals = st["surv_verts"] + K2 * st["surv_edges"]
    res.update(narrow_fwd_ms=round(k_ms, 3), sdf_evaluations=int(evals),
               sdf_evaluations_per_s=round(evals / (k_ms * 1e-3), 1))
    log("prims leg %s" % res)
    del plan, ctx
    torch.cuda.empty_cache()
    return res


def golden_c4():
    """Stored FP64 oracle values of sampled queries of the large workload."""
    path = os.path.join(HERE, "tests", "golden", "c4_oracle.json")
    with open(path) as f:
        return json.load(f)


def parity_of(g_gpu, grad, hv, ref_groups, ref_grad, ref_hv, Ls_groups):
    pos = np.abs(g_gpu[:, [0, 1, 2, 6, 7, 8, 9]] - ref_groups[:, [0, 1, 2, 6, 7, 8, 9]]).max(1) / Ls_groups
    out = {"max_pos_err_over_Ls": float(pos.max())}
    if ref_grad is not None:
        gerr = np.linalg.norm(grad - ref_grad, axis=1) / np.maximum(np.linalg.norm(ref_grad, axis=1), 1e-30)
        herr = np.linalg.norm(hv - ref_hv, axis=1) / np.maximum(np.linalg.norm(ref_hv, axis=1), 1e-30)
        out.update(max_grad_rel_err=float(gerr.max()), max_hvp_rel_err=float(herr.max()))
    return out


def step_leg(api, W, config, pairs, budget_gb, args, steps, warmup, golden=None, quick=False):
    """One workload: objects resident, one plan, autotuned launch shape, `warmup`
    untimed and `steps` timed cm_contacts_step calls.  Returns a dict of figures
    and the live objects for the legs that follow."""
    import torch
    w = build_workload(config, pairs)
    log("workload %s: %d pair-queries, %d objects" % (config, w.n, len(w.objects)))
    ctx = api.Context(0, L_ref=w.L_ref, budget_bytes=int(budget_gb * (1 << 30)),
                      prune_pieces=0 if args.no_prune else 1)
    hs = ctx.build_objects(w.objects)
    torch.cuda.synchronize()
    log("objects resident")
    plan = ctx.plan(hs[w.qa], hs[w.qb])
    log("plan: %d groups, %d contacts" % (plan.G, plan.C))
    qd = plan.device_queries(w.poses)
    cot = W.cotangents(w.cot_seed or 1, plan.G)
    direc = W.directions(w.cot_seed or 1, w.n)
    if golden is not None:
        # the stored oracle values were taken with these cotangents and directions
        goff_s = np.array(golden["group_off"], np.int64)
        cot_s = W.cotangents(golden["workload"]["cot_seed"], goff_s[-1])
        dir_s = W.directions(golden["workload"]["cot_seed"], len(golden["sel"]))
        for k, i in enumerate(golden["sel"]):
            assert plan.group_off[i + 1] - plan.group_off[i] == goff_s[k + 1] - goff_s[k]
            cot[plan.group_off[i]:plan.group_off[i + 1]] = cot_s[goff_s[k]:goff_s[k + 1]]
            direc[i] = dir_s[k]
    cot_d = torch.tensor(np.ascontiguousarray(cot.T, np.float32)).cuda()
    dir_d = torch.tensor(direc.astype(np.float32)).cuda()
    out = torch.empty((12, plan.G), dtype=torch.float32, device="cuda")
    grad = torch.empty((w.n, 12), dtype=torch.float32, device="cuda")
    grad2 = torch.empty_like(grad)
    hv = torch.empty_like(grad)
    stream = torch.cuda.current_stream()

    def step():
        plan.step(qd, cot_d, dir_d, out=out, grad=grad, hv=hv, stream=stream)

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
        if args.wg_waves:
            plan.wg_waves = tuple(int(v) for v in args.wg_waves.split(","))
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
        plan.wg_waves = tp.wg_waves
        del tp, tq, tc, tg
        tuned_on = ns
    how = ("autotuned on %d pair-queries" % tuned_on) if tuned_on else "set by --launch-shape"
    log("launch shape (%s): %d workgroups per CU of %d waves (dual sweeps), %d of %d (float sweeps)"
        % (how, shape, plan.wg_waves[1], shape_f, plan.wg_waves[0]))
    long_steps = config == "c4"  # seconds per step: report each one
    for k in range(warmup):
        step()
        if long_steps:
            torch.cuda.synchronize()
            log("warmup step %d/%d" % (k + 1, warmup))
    torch.cuda.synchronize()
    log("warmup done")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.time()
    e0.record(stream)
    for k in range(steps):
        step()
        if long_steps:
            torch.cuda.synchronize()
            log("timed step %d/%d" % (k + 1, steps))
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.time() - t_wall
    ms = e0.elapsed_time(e1) / steps
    log("timed %d steps: %.2f ms/step (wall %.2f s)" % (steps, ms, wall))
    # the step's outputs (every timed step gives the same), kept apart from the
    # buffers the other legs reuse
    step_out = (out.clone(), grad.clone(), hv.clone())
    res = dict(w=w, ctx=ctx, hs=hs, plan=plan, qd=qd, cot=cot, direc=direc, cot_d=cot_d, dir_d=dir_d,
               out=out, grad=grad, hv=hv, ms=ms, wall=wall, shape=shape, shape_f=shape_f, tuned_on=tuned_on,
               wg_waves=plan.wg_waves,
               step=step, timed=timed, stream=stream, step_out=step_out)
    # the step's outputs now are those of every timed step (deterministic launches)
    if golden is not None:
        sel = np.array(golden["sel"], np.int64)
        rows = np.concatenate([np.arange(plan.group_off[i], plan.group_off[i + 1]) for i in sel])
        goff_s = np.array(golden["group_off"], np.int64)
        Ls = np.repeat(np.array(golden["scene_scale"]), np.diff(goff_s))
        g_gpu = out.cpu().numpy().T.astype(np.float64)[rows]
        gr_gpu = grad.cpu().numpy()[sel].astype(np.float64)
        hv_gpu = hv.cpu().numpy()[sel].astype(np.float64)
        res["parity"] = dict(queries=len(sel), source="tests/golden/c4_oracle.json (FP64 oracle)",
                             **parity_of(g_gpu, gr_gpu, hv_gpu, np.array(golden["records"]),
                                         np.array(golden["grad"]), np.array(golden["hv"]), Ls))
        # the acceptance bounds of the parity tests: 1e-4 relative (floor 1e-3 |cot| max(1, L_s)),
        # or 4 times the oracle's FP32 spread where a query is ill-conditioned at FP32
        cq = np.sqrt(np.add.reduceat((cot_s.astype(np.float64) ** 2).sum(1), goff_s[:-1]))
        floor = 1e-3 * cq * np.maximum(1.0, np.array(golden["scene_scale"]))
        for name, got, key in (("grad", gr_gpu, "grad"), ("hvp", hv_gpu, "hv")):
            ref = np.array(golden[key])
            allowed = np.maximum(1e-4 * np.maximum(np.linalg.norm(ref, axis=1), floor),
                                 4.0 * np.array(golden["spread_" + key]))
            res["parity"]["max_%s_err_over_allowed" % name] = float(
                (np.linalg.norm(got - ref, axis=1) / allowed).max())
        # positions within 1e-5 L_s, derivatives within their bounds: the headline's accuracy condition
        res["parity"]["within_bounds"] = bool(res["parity"]["max_pos_err_over_Ls"] <= 1e-5 and
                                              res["parity"]["max_grad_err_over_allowed"] <= 1.0 and
                                              res["parity"]["max_hvp_err_over_allowed"] <= 1.0)
        log("parity against the stored oracle values: %s" % res["parity"])
    if quick:
        return res
    # the forward + gradient step, the forward pass, and the step from its HIP graph
    reps = 1 if long_steps else 2
    sep_ms = None
    if not args.no_separate and not long_steps:
        def separate():
            plan.forward(qd, out=out, stream=stream)
            plan.backward(qd, cot_d, grad=grad2, stream=stream)
            plan.hvp(qd, cot_d, dir_d, hv=hv, grad=grad2, stream=stream)
        sep_ms = timed(separate, reps)
    fg_ms = timed(lambda: plan.step(qd, cot_d, out=out, grad=grad2, stream=stream), reps)
    fw_ms = timed(lambda: plan.forward(qd, out=out, stream=stream), reps)
    log("separate calls %s ms, forward + gradient step %.2f ms, forward %.2f ms" % (sep_ms, fg_ms, fw_ms))
    graph = plan.graph(qd, cot_d, grad, dir_d, hv, out)
    graph_ms = timed(lambda: graph.launch(stream), 1 if long_steps else max(steps, 2))
    del graph
    log("graph replay %.2f ms" % graph_ms)
    res.update(sep_ms=sep_ms, fg_ms=fg_ms, fw_ms=fw_ms, graph_ms=graph_ms)
    # per-kernel timing of the step (events on the launch stream), untimed region
    plan.set_timing(True)
    step()
    torch.cuda.synchronize()
    tk = plan.timing()
    plan.set_timing(False)
    work_v, work_e = plan.work()
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
    res["split"] = {k: round(v, 3) for k, v in tk.items() if v >= 0}
    res["stats"] = st
    res["roofline"] = {
        "bound": "alu", "kernel": "k_narrow<df, forward, tape>", "achieved": round(achieved / 1e12, 3),
        "peak": round(PEAK_LANE_OPS / 1e12, 3), "unit": "T lane-op/s (FP32 VALU)",
        "frac": round(achieved / PEAK_LANE_OPS, 4), "traffic": measured_traffic(config, w.n),
        "kernel_ms": round(dom_ms, 3), "alg_ops_per_launch": int(alg_ops),
        "algorithmic_point_plane": int(st["pairs"]), "performed_point_plane": int(work_v + work_e),
        "performed_achieved": round(perf_achieved / 1e12, 3),
        "performed_frac": round(perf_achieved / PEAK_LANE_OPS, 4)}
    log("roofline %s" % res["roofline"])
    # the forward pass alone (records only): its narrow-phase kernel against the same peak
    plan.set_timing(True)
    plan.forward(qd, out=out, stream=stream)
    torch.cuda.synchronize()
    fwd_k = plan.timing()["narrow_fwd"]
    fwork_v, fwork_e = plan.work()
    plan.set_timing(False)
    fv, fe = OPS["forward"]
    f_ops = st["vertex_pairs"] * fv + st["edge_pairs"] * fe
    f_perf = fwork_v / max(st["vertex_pairs"], 1) * st["vertex_pairs"] * fv + \
        fwork_e / max(st["edge_pairs"] * (2 * K_TRACE + 1), 1) * st["edge_pairs"] * fe
    res["forward_roofline"] = {
        "bound": "alu", "kernel": "k_narrow<float, forward>", "kernel_ms": round(fwd_k, 3),
        "achieved": round(f_ops / (fwd_k * 1e-3) / 1e12, 3), "unit": "T lane-op/s (FP32 VALU)",
        "frac": round(f_ops / (fwd_k * 1e-3) / PEAK_LANE_OPS, 4), "alg_ops_per_launch": int(f_ops),
        "performed_frac": round(f_perf / (fwd_k * 1e-3) / PEAK_LANE_OPS, 4)}
    log("forward roofline %s" % res["forward_roofline"])
    # plain per-pair launch: same kernels, one pair-query per launch
    if not args.no_plain:
        ns = min(args.plain_sample or (16 if long_steps else 64), w.n)
        plans = []
        for i in range(ns):
            p1 = ctx.plan(hs[w.qa[i:i + 1]], hs[w.qb[i:i + 1]])
            p1.launch_shape = plan.launch_shape
            p1.wg_waves = plan.wg_waves
            q1 = p1.device_queries(w.poses[i:i + 1])
            g0, g1 = plan.group_off[i], plan.group_off[i + 1]
            c1 = cot_d[:, g0:g1].contiguous()
            o1 = torch.empty((12, p1.G), dtype=torch.float32, device="cuda")
            gr1 = torch.empty((1, 12), dtype=torch.float32, device="cuda")
            plans.append((p1, q1, c1, dir_d[i:i + 1].contiguous(), o1, gr1, torch.empty_like(gr1)))

        def plain_pass():
            for p1, q1, c1, d1, o1, gr1, hv1 in plans:
                p1.step(q1, c1, d1, out=o1, grad=gr1, hv=hv1, stream=stream)

        pms = timed(plain_pass, 1)
        # the plain launches give the same results as the batched step (bitwise)
        so, sg, sh = step_out
        same = all(torch.equal(o1, so[:, plan.group_off[i]:plan.group_off[i + 1]]) and torch.equal(gr1[0], sg[i])
                   and torch.equal(hv1[0], sh[i]) for i, (p1, q1, c1, d1, o1, gr1, hv1) in enumerate(plans))
        step()
        torch.cuda.synchronize()
        res["plain"] = {"sample": ns, "ms": round(pms, 3), "value": round(ns / (pms * 1e-3), 1),
                        "unit": "pair-queries/s", "bitwise_equal_to_batched": bool(same),
                        "note": "first %d pair-queries, one cm_contacts_step (records + gradient + H v) per query, "
                                "same kernels and launch shape" % ns}
        log("plain launch %s" % res["plain"])
        del plans
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c4", choices=["c0", "c1", "c2", "c4"])
    ap.add_argument("--pairs", type=int, default=None, help="batch size override (default: the config's)")
    ap.add_argument("--budget-gb", type=float, default=None, help="device-memory budget (default per workload)")
    ap.add_argument("--no-prune", action="store_true", help="evaluate every piece (no piece pruning)")
    ap.add_argument("--plain-sample", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="skip the secondary (16384-pair) step figure")
    ap.add_argument("--no-separate", action="store_true", help="skip timing the three separate calls")
    ap.add_argument("--no-tight", action="store_true", help="skip the step with the tighter edge bound")
    ap.add_argument("--launch-shape", default=None,
                    help="F,D: fixed persistent workgroups per CU for the float and dual sweeps (no autotuning)")
    ap.add_argument("--wg-waves", default=None,
                    help="F,D: waves per workgroup for the float and dual sweeps (with --launch-shape)")
    ap.add_argument("--tune-sample", type=int, default=16384,
                    help="autotune on a plan of the first N pair-queries when the batch is larger")
    ap.add_argument("--sweep", action="store_true",
                    help="only the broad-phase sweep (broad + narrow vs narrow only over d_max); prints its own JSON line")
    ap.add_argument("--no-spline", action="store_true", help="skip the spline-representation leg")
    ap.add_argument("--no-prims", action="store_true", help="skip the primitive-representation leg")
    ap.add_argument("--curve-study", action="store_true",
                    help="only the serialization study (no curve / Morton / Hilbert); prints its own JSON line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device copy of 1 GiB three times (scale of the HBM traffic counters)")
    ap.add_argument("--serve-rates", default="2000,5000,10000,20000", help="Poisson request rates (req/s)")
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--cpu-child", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_child:
        with open(args.cpu_child) as f:
            spec = json.load(f)
        os.unlink(args.cpu_child)
        cpu_child(spec)
        return
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
    if args.curve_study:
        print(json.dumps({"curve_study": curve_study_leg()}), flush=True)
        return

    cfg = args.config
    golden = golden_c4() if cfg == "c4" and args.pairs in (None, 65536) else None
    budget_gb = args.budget_gb or BUDGET_GB[cfg]
    # the oracle leg runs in a child process while the GPU legs run; it needs
    # the cotangents and directions, which depend only on the workload's seeds
    child = None
    if not args.no_cpu_baseline:
        wl = build_workload(cfg, args.pairs)
        # groups of the queries the oracle samples (the cotangents are a prefix of the batch's)
        n_groups = int(sum(wl.objects[a].n_pieces + wl.objects[b].n_pieces
                           for a, b in zip(wl.qa[:CPU_SAMPLE[cfg][0]], wl.qb[:CPU_SAMPLE[cfg][0]])))
        threads = max(1, min(os.cpu_count() or 1, 16) - 1)
        child = start_cpu_child(cfg, args.pairs, W.cotangents(wl.cot_seed or 1, n_groups),
                                W.directions(wl.cot_seed or 1, wl.n), threads)
        del wl
    r = step_leg(api, W, cfg, args.pairs, budget_gb, args, args.steps, args.warmup, golden=golden)
    w, plan = r["w"], r["plan"]
    ms = r["ms"]

    # the same step with the tighter edge bound of the broad phase (outputs are
    # unchanged, only the candidate lists shrink), in a context of its own
    tight = None
    if not args.no_tight and cfg != "c4":  # (c4: a second plan would double its scratch)
        ctx_t = api.Context(0, L_ref=w.L_ref, budget_bytes=int(budget_gb * (1 << 30)), edge_bound=1)
        hs_t = ctx_t.build_objects(w.objects)
        plan_t = ctx_t.plan(hs_t[w.qa], hs_t[w.qb])
        plan_t.launch_shape = plan.launch_shape
        plan_t.wg_waves = plan.wg_waves
        qd_t = plan_t.device_queries(w.poses)
        o_t, g_t, h_t = torch.empty_like(r["out"]), torch.empty_like(r["grad"]), torch.empty_like(r["hv"])
        t_ms = r["timed"](lambda: plan_t.step(qd_t, r["cot_d"], r["dir_d"], out=o_t, grad=g_t, hv=h_t,
                                              stream=r["stream"]), max(args.steps, 2))
        st_t = plan_t.stats()
        tight = {"ms_per_step": round(t_ms, 3), "value": round(w.n / (t_ms * 1e-3), 1),
                 "surviving_contacts": st_t["surv_verts"] + st_t["surv_edges"],
                 "note": "edge bound max(max(lb1, lb2) - l, (lb1 + lb2 - l) / 2) instead of min(lb1, lb2) - l"}
        log("tight edge bound %s" % tight)
        del plan_t, qd_t, ctx_t, o_t, g_t, h_t

    out_h = r["step_out"][0].cpu().numpy().T.astype(np.float64)
    grad_h = r["step_out"][1].cpu().numpy().astype(np.float64)
    hv_h = r["step_out"][2].cpu().numpy().astype(np.float64)
    config_line = {"workload": "%s: %d pair-queries, forward + gradient (both poses) + HVP per step" % (cfg, w.n),
                   "pair_queries": w.n, "groups": plan.G, "contacts": plan.C, "step": "cm_contacts_step",
                   "budget_gb": budget_gb}
    if cfg == "c4":
        config_line["objects"] = "library of 2048 (32 pieces, hulls of log-uniform [64, 1024] points)"
    line_extra = dict(
        split_ms=r["split"], separate_calls_ms_per_step=round(r["sep_ms"], 3) if r["sep_ms"] else None,
        graph_replay_ms_per_step=round(r["graph_ms"], 3),
        launch_shape={"workgroups_per_cu": r["shape"], "workgroups_per_cu_float": r["shape_f"],
                      "waves_per_workgroup": r["wg_waves"][1], "waves_per_workgroup_float": r["wg_waves"][0],
                      "tile": "one wave of 64 contacts", "tuned_on_pair_queries": r["tuned_on"]},
        forward_gradient_step_ms=round(r["fg_ms"], 3), forward_gradient_value=round(w.n / (r["fg_ms"] * 1e-3), 1),
        forward_ms=round(r["fw_ms"], 3), forward_value=round(w.n / (r["fw_ms"] * 1e-3), 1),
        forward_roofline=r["forward_roofline"], tight_edge_bound=tight, work=r["stats"])
    parity = r.get("parity")
    plain = r.get("plain")
    roofline = r["roofline"]
    radii = np.array([o.radius() for o in w.objects])
    del r, plan
    torch.cuda.empty_cache()

    # the secondary figure: the same step on the 16384-pair differentiation workload
    secondary = None
    if cfg == "c4" and not args.no_secondary:
        r2 = step_leg(api, W, "c2", None, BUDGET_GB["c2"], args, 5, 2, quick=True)
        secondary = {"workload": "c2: 16384 pair-queries (log-uniform [1, 32] pieces of [8, 512] points)",
                     "ms_per_step": round(r2["ms"], 3), "value": round(r2["w"].n / (r2["ms"] * 1e-3), 1),
                     "launch_shape": [r2["shape_f"], r2["shape"]]}
        log("secondary %s" % secondary)
        del r2
        torch.cuda.empty_cache()

    spline = None
    if not args.no_spline:
        spline = spline_leg()
    prims = None
    if not args.no_prims:
        prims = prims_leg()

    serving = None
    if not args.no_serving:
        serving = serving_leg(api, W, [float(x) for x in args.serve_rates.split(",")], args.serve_seconds)
        log("serving %s" % serving)

    cpu = None
    if child is not None:
        spec = child[1]
        outs, _ = child[0].communicate(timeout=900)
        res = json.loads(outs.strip().splitlines()[-1])
        ns = res["n"]
        what = "forward + hyper-dual gradient and HVP" if spec["grad"] else "forward records only"
        cpu = {"value": round(ns / res["seconds"], 4), "unit": "pair-queries/s", "cores": spec["threads"],
               "kind": "oracle",
               "sample": "first %d pair-queries of the workload, FP64 %s, OpenMP over queries (%.1f s; building "
                         "their objects' hulls and grids took %.1f s more)" % (ns, what, res["seconds"],
                                                                               res["objects_s"])}
        goff = np.array(res["goff"], np.int64)
        Ls = np.repeat(radii[w.qa[:ns]] + radii[w.qb[:ns]], np.diff(goff))
        po = parity_of(out_h[: goff[-1]], grad_h[:ns], hv_h[:ns], np.array(res["groups"]),
                       np.array(res["grad"]) if "grad" in res else None,
                       np.array(res["hv"]) if "hv" in res else None, Ls)
        po["queries"] = ns
        po["source"] = "oracle run here"
        parity = {"stored": parity, "here": po} if parity is not None else po
        log("cpu baseline %s parity %s" % (cpu, po))

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
        "config": config_line,
    }
    line.update(line_extra)
    line.update({"roofline": roofline, "cpu_baseline": cpu, "plain_launch": plain, "parity": parity,
                 "secondary": secondary, "spline": spline, "prims": prims, "serving": serving})
    if plain:
        line["vs_plain_launch"] = round(value / plain["value"], 2)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
