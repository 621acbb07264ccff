"""Writes c4_oracle.json beside this file: the FP64 oracle's results for four
pair-queries sampled from the large workload (65536 pairs of 32-piece objects,
pieces hulls of log-uniform [64, 1024] ellipsoid points, the objects drawn
from a library of 2048), so that the GPU test of the full launch can compare
against them without re-running the oracle (about 11 minutes of hyper-dual
arithmetic per query on one core).

Stored per sampled query: the group records (p, n, d, q, W, logZ), the gradient
of <c, records> w.r.t. both poses and the Hessian-vector product along the
query's direction, the FP32 spread of both (oracle.fp32_spread, seeds 1 and 2)
and the scene scale r_A + r_B.  The cotangents and directions are the seeded
ones of paper_2604_17538_amd.workloads (cotangents over the sampled queries'
groups in order, as for the other parity tests), and a digest of the sampled
inputs lets the test check that it regenerated the same workload.

Only the oracle and the seeded input generators are called.  Usage:
    python tests/golden/c4_oracle.py [--threads 4]
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
N_SAMPLE = 4
SEEDS = (1, 2)
OUT = os.path.join(HERE, "c4_oracle.json")


def sample(n):
    return np.linspace(0, n - 1, N_SAMPLE).astype(np.int64)


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=N_SAMPLE)
    args = ap.parse_args()
    import oracle as O
    from paper_2604_17538_amd import workloads as W
    O.build(force=False)
    t0 = time.time()
    w = W.config4(n_envs=N_ENVS, library=LIBRARY)
    sel = sample(w.n)
    prm = O.default_params(w.L_ref)
    need = sorted({int(w.qa[i]) for i in sel} | {int(w.qb[i]) for i in sel})

    def make(j):
        o = O.from_workload_object(w.objects[j])
        o.build_grid(prm)
        return j, o

    objs = [None] * len(w.objects)
    with ThreadPoolExecutor(len(need)) as ex:
        for j, o in ex.map(make, need):
            objs[j] = o
    print("objects %.1f s" % (time.time() - t0), flush=True)
    qa, qb, poses = w.qa[sel], w.qb[sel], w.poses[sel]
    g, goff = O.contacts(prm, objs, qa, qb, poses, threads=args.threads)
    print("records %.1f s" % (time.time() - t0), flush=True)
    cot = W.cotangents(w.cot_seed, goff[-1])
    direc = W.directions(w.cot_seed, len(sel))
    dg, dh, grad, hv = O.fp32_spread(prm, objs, qa, qb, poses, cot, direc, seeds=SEEDS, threads=args.threads,
                                     concurrent=True, return_base=True)
    print("gradient, H v and spread %.1f s" % (time.time() - t0), flush=True)
    r = np.array([objs[j].radius() if objs[j] is not None else 0.0 for j in range(len(objs))])
    doc = {
        "workload": {"n_envs": N_ENVS, "library": LIBRARY, "seed": W.SEED_BASE + 4, "cot_seed": int(w.cot_seed)},
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
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=0)
    print("wrote %s (%.1f s)" % (OUT, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
