"""Helpers shared by the GPU parity tests: contact matching between the HIP
path's (serialized) geometry order and the oracle's order, and the tolerance
checks of the acceptance criteria:

* positions and distances (p, q, d, tau_b logZ, per-contact p_c and d_c):
  |delta| <= 1e-5 * L_s, L_s = r_A + r_B;
* weights and W: |delta| <= 1e-4 * w where w >= 1e-6, else <= 1e-10;
* normals: |delta n| <= 1e-4 where |m| >= 1e-3 (m = sum_i w_i n_c,i);
* candidate lists (broad-phase masks): equal except for contacts whose oracle
  bound is within 1e-6 of d_max or whose point is within 1e-6 of a voxel face.

Where a record is ill-conditioned at FP32 precision -- the oracle's probe,
which perturbs every intermediate an FP32 evaluation rounds by one rounding,
already moves it by more than its bound (a blended W made of contacts in the
transition band, where f = s^3 (...) turns a tiny change of phi into a large
relative change of f) -- the bound of that component is K_SPREAD times that
spread, as for the derivatives.
"""
import numpy as np

POS_TOL = 1e-5
REL_TOL = 1e-4
W_FLOOR = 1e-6
BAND = 1e-6


def contact_perm(ex: dict, ob) -> np.ndarray:
    """perm[i] = oracle-local contact index of the HIP path's object-local contact i.

    Both sides list, per piece, its vertices then its edges; vertices are matched
    by exact coordinates (both come from the same input points), edges by their
    endpoint pair."""
    perm = []
    obase = 0
    for k in range(len(ex["vert_off"]) - 1):
        pv = ex["verts"][ex["vert_off"][k]:ex["vert_off"][k + 1]]
        ov = ob.verts[ob.vert_off[k]:ob.vert_off[k + 1]]
        pe = ex["edges"][ex["edge_off"][k]:ex["edge_off"][k + 1]]
        oe = ob.edges[ob.edge_off[k]:ob.edge_off[k + 1]]
        assert len(pv) == len(ov) and len(pe) == len(oe), "piece %d: vertex/edge counts differ" % k
        omap = {tuple(v): j for j, v in enumerate(ov)}
        vmap = np.array([omap[tuple(v)] for v in pv])
        emap = {tuple(sorted(e)): j for j, e in enumerate(oe)}
        perm.extend(obase + vmap)
        perm.extend(obase + len(ov) + np.array([emap[tuple(sorted((vmap[a], vmap[b])))] for a, b in pe], int))
        obase += len(ov) + len(oe)
    return np.array(perm, np.int64)


def query_contact_perm(perm_obj, qa, qb, coff_o):
    """Global permutation HIP contact index -> oracle contact index for a batch."""
    out = []
    for i, (a, b) in enumerate(zip(qa, qb)):
        pa, pb = perm_obj[a], perm_obj[b]
        out.append(coff_o[i] + pa)
        out.append(coff_o[i] + len(pa) + pb)
    return np.concatenate(out)


K_SPREAD = 4.0


def check_groups(g_gpu: np.ndarray, g_or: np.ndarray, Ls: np.ndarray, tau_b: float, m_or=None, spread=None):
    """g_gpu [G,12] and g_or [G,12]; Ls [G] scene scale per group; spread
    (optional, [G,12]) the oracle's FP32 spread of each record component.
    Returns a dict of worst normalised errors (<= 1 passes)."""
    sp = np.zeros_like(g_or) if spread is None else K_SPREAD * np.asarray(spread)
    pos_cols = [0, 1, 2, 6, 7, 8, 9]
    pos = (np.abs(g_gpu[:, pos_cols] - g_or[:, pos_cols]) / np.maximum(POS_TOL * Ls[:, None], sp[:, pos_cols])).max(1)
    lz = np.abs(tau_b * (g_gpu[:, 11] - g_or[:, 11])) / np.maximum(POS_TOL * Ls, tau_b * sp[:, 11])
    W = g_or[:, 10]
    dW = np.abs(g_gpu[:, 10] - W)
    wn = np.where(W >= W_FLOOR, dW / np.maximum(REL_TOL * np.maximum(W, 1e-30), sp[:, 10]),
                  dW / np.maximum(1e-10, sp[:, 10]))
    if m_or is None:
        nmask = np.ones(len(g_or), bool)
    else:
        nmask = np.linalg.norm(m_or, axis=1) >= 1e-3
    dn = (np.abs(g_gpu[:, 3:6] - g_or[:, 3:6]) / np.maximum(REL_TOL, sp[:, 3:6])).max(1)
    dn = np.where(nmask, dn, 0.0)
    return dict(pos=pos.max(initial=0), logZ=lz.max(initial=0), W=wn.max(initial=0), n=dn.max(initial=0),
                argpos=int(np.argmax(pos)) if len(pos) else -1)
