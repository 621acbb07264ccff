"""Writes c4_oracle.json beside this file: the FP64 oracle's results for
pair-queries sampled from the large workload (65536 pairs of 32-piece objects,
pieces hulls of log-uniform [64, 1024] ellipsoid points, the objects drawn
from a library of 2048), so that the GPU test of the full launch can compare
against them without re-running the oracle (several minutes of hyper-dual
arithmetic per query on one core).

Which queries: the oracle's own forward records of N_CANDIDATES evenly spaced
queries decide.  A query's active groups are those with blended Jacobian
weight W > 1e-6 (some contact within d_max); the N_ACTIVE queries with the most
active groups are kept, then up to N_SHALLOW more whose deepest group is near
contact only (0 <= min d < d_max), then the deepest remaining query, so the
sample holds deep penetration, near contact and fully filtered pieces.

Stored per sampled query: the group records (p, n, d, q, W, logZ), the gradient
of <c, records> w.r.t. both poses and the Hessian-vector product along the
query's direction, the FP32 spread of both (oracle.fp32_spread, seeds 1 and 2)
and the scene scale r_A + r_B.  The cotangents and directions are the seeded
ones of paper_2604_17538_amd.workloads (cotangents over the sampled queries'
groups in order, as for the other parity tests), and a digest of the sampled
inputs lets the test check that it regenerated the same workload.

Also stored: the FP32 spread of every record component (the change of the
records when every intermediate an FP32 evaluation rounds is perturbed by one
rounding, oracle seeds 1, 2 and 3; the max over seeds): a blended W made of
contacts in the transition band moves by far more than 1e-4 of itself under
such perturbations, so no FP32 evaluation can be held tighter there.

Only the oracle and the seeded input generators are called.  Usage:
    python tests/golden/c4_oracle.py [--threads 8]
    python tests/golden/c4_oracle.py --record-spread   (adds the record spread
        to an existing c4_oracle.json of the same workload)
"""
import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

N_ENVS = 65536
LIBRARY = 2048
N_CANDIDATES = 32
N_ACTIVE = 8
N_SHALLOW = 2
SEEDS = (1, 2)
W_ACTIVE = 1e-6
OUT = os.path.join(HERE, "c4_oracle.json")


def candidates(n):
    return np.linspace(0, n - 1, N_CANDIDATES).astype(np.int64)


def input_digest(w, sel):
    """sha256 over the sampled queries' poses and their objects' points."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(w.poses[sel], np.float64).tobytes())
    for i in sel:
        for j in (int(w.qa[i]), int(w.qb[i])):
            o = w.objects[j]
            h.update(np.ascontiguousarray(o.points, np.float64).tobytes())
            h.update(np.ascontiguousarray(o.offsets, np.int64).tobytes())
    return h.hexdigest()


def choose(cand, g, goff, d_max):
    """Indices into cand of the sampled queries (rule in the module docstring)."""
    act, dmin = [], []
    for k in range(len(cand)):
        G = g[goff[k]:goff[k + 1]]
        act.append(int((G[:, 10] > W_ACTIVE).sum()))
        dmin.append(float(G[:, 6].min()))
    act, dmin = np.array(act), np.array(dmin)
    order = sorted(range(len(cand)), key=lambda k: (-act[k], k))
    pick = [k for k in order if act[k] > 0][:N_ACTIVE]
    shallow = [k for k in range(len(cand)) if k not in pick and 0.0 <= dmin[k] < d_max - 1e-12]
    pick += shallow[:N_SHALLOW]
    rest = [k for k in range(len(cand)) if k not in pick]
    if rest:
        pick.append(min(rest, key=lambda k: dmin[k]))
    pick = sorted(pick)
    return np.array(pick, np.int64), act, dmin


REC_SEEDS = (1, 2, 3)


def record_spread(O, prm, objs, qa, qb, poses, threads):
    """Per group and component, the largest change of the records over the
    probe seeds (max |records(seed) - records|), [G, 12]."""
    g0, _ = O.contacts(prm, objs, qa, qb, poses, threads=threads)
    sp = np.zeros_like(g0)
    for s in REC_SEEDS:
        p = O.Params.from_buffer_copy(prm)
        p.jitter, p.jitter_seed = O.FP32_UNIT_ROUNDOFF, int(s)
        g, _ = O.contacts(p, objs, qa, qb, poses, threads=threads)
        sp = np.maximum(sp, np.abs(g - g0))
    return g0, sp


def add_record_spread(threads):
    import oracle as O
    from paper_2604_17538_amd import workloads as W
    O.build(force=False)
    with open(OUT) as f:
        doc = json.load(f)
    w = W.config4(n_envs=N_ENVS, library=LIBRARY)
    sel = np.array(doc["sel"], np.int64)
    assert input_digest(w, sel) == doc["input_sha256"]
    prm = O.default_params(w.L_ref)
    objs = [None] * len(w.objects)
    for j in sorted({int(w.qa[i]) for i in sel} | {int(w.qb[i]) for i in sel}):
        objs[j] = O.from_workload_object(w.objects[j])
        objs[j].build_grid(prm)
    g0, sp = record_spread(O, prm, objs, w.qa[sel], w.qb[sel], w.poses[sel], threads)
    assert np.array_equal(g0, np.array(doc["records"])), "the oracle no longer gives the stored records"
    doc["spread_records"] = sp.tolist()
    doc["record_spread_seeds"] = list(REC_SEEDS)
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=0)
    print("added the record spread to %s" % OUT, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("--record-spread", action="store_true")
    args = ap.parse_args()
    if args.record_spread:
        add_record_spread(args.threads)
        return
    import oracle as O
    from paper_2604_17538_amd import workloads as W
    O.build(force=False)
    t0 = time.time()
    w = W.config4(n_envs=N_ENVS, library=LIBRARY)
    cand = candidates(w.n)
    prm = O.default_params(w.L_ref)
    need = sorted({int(w.qa[i]) for i in cand} | {int(w.qb[i]) for i in cand})

    def make(j):
        o = O.from_workload_object(w.objects[j])
        o.build_grid(prm)
        return j, o

    objs = [None] * len(w.objects)
    with ThreadPoolExecutor(2) as ex:
        for j, o in ex.map(make, need):
            objs[j] = o
    print("objects %.1f s" % (time.time() - t0), flush=True)
    gc, goc = O.contacts(prm, objs, w.qa[cand], w.qb[cand], w.poses[cand], threads=args.threads)
    pick, act, dmin = choose(cand, gc, goc, prm.d_max)
    sel = cand[pick]
    print("candidates %.1f s; selected %s (active groups %s, min d %s)"
          % (time.time() - t0, sel.tolist(), act[pick].tolist(), np.round(dmin[pick], 5).tolist()), flush=True)
    qa, qb, poses = w.qa[sel], w.qb[sel], w.poses[sel]
    g, goff = O.contacts(prm, objs, qa, qb, poses, threads=args.threads)
    cot = W.cotangents(w.cot_seed, goff[-1])
    direc = W.directions(w.cot_seed, len(sel))
    dg, dh, grad, hv = O.fp32_spread(prm, objs, qa, qb, poses, cot, direc, seeds=SEEDS,
                                     threads=max(1, args.threads // (len(SEEDS) + 1)),
                                     concurrent=True, return_base=True)
    print("gradient, H v and spread %.1f s" % (time.time() - t0), flush=True)
    _, rsp = record_spread(O, prm, objs, qa, qb, poses, args.threads)
    r = np.array([objs[j].radius() if objs[j] is not None else 0.0 for j in range(len(objs))])
    doc = {
        "workload": {"n_envs": N_ENVS, "library": LIBRARY, "seed": W.SEED_BASE + 4, "cot_seed": int(w.cot_seed)},
        "selection": {"candidates": cand.tolist(), "active_groups": act.tolist(), "min_d": dmin.tolist(),
                      "rule": "most active groups (W > 1e-6), then near-contact-only, then the deepest remaining"},
        "sel": sel.tolist(),
        "input_sha256": input_digest(w, sel),
        "group_off": goff.tolist(),
        "records": g.tolist(),
        "grad": grad.tolist(),
        "hv": hv.tolist(),
        "spread_grad": dg.tolist(),
        "spread_hv": dh.tolist(),
        "scene_scale": (r[qa] + r[qb]).tolist(),
        "spread_seeds": list(SEEDS),
        "spread_records": rsp.tolist(),
        "record_spread_seeds": list(REC_SEEDS),
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=0)
    print("wrote %s (%.1f s)" % (OUT, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
