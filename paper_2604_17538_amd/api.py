"""Python API over the C ABI (include/cm.h): contexts, resident objects, plans,
launches on torch-managed device memory and streams, and the autograd layer
(ContactFn) whose backward passes call the library's adjoint, Hessian-vector
and Jacobian-vector entry points.

PyTorch provides device memory, streams and the autograd graph only; every
step of the contact pipeline and its derivatives runs in libcm.so's gfx950
kernels.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

from . import _cm
from ._cm import cm_groups, cm_params, QUERY_DTYPE


class CMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_cm.STATUS_NAMES.get(status, str(status)), msg))
        self.status = status


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def default_params(L_ref: float = 0.1, **overrides) -> cm_params:
    p = cm_params()
    st = _cm.cm_default_params(float(L_ref), ctypes.byref(p))
    if st != 0:
        raise CMError(st, "cm_default_params")
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def _torch():
    import torch
    return torch


def _stream_ptr(stream) -> ctypes.c_void_p:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """A device context owning resident geometry (device=-1: host-only)."""

    def __init__(self, device: int = 0, params: Optional[cm_params] = None, L_ref: float = 0.1,
                 budget_bytes: int = 0, **overrides):
        self.params = params if params is not None else default_params(L_ref, **overrides)
        if device >= 0:
            # let torch bring up the device first: it shares the HIP runtime with
            # the library and must own the device's initialisation
            _torch().cuda.init()
        self._h = ctypes.c_void_p()
        st = _cm.cm_init(int(device), ctypes.byref(self.params), int(budget_bytes), ctypes.byref(self._h))
        if st != 0:
            raise CMError(st, "cm_init(device=%d)" % device)
        self.device = device

    @property
    def handle(self):
        return self._h

    def _check(self, st, what):
        if st != 0:
            raise CMError(st, "%s: %s" % (what, _cm.cm_last_error(self._h).decode()))

    def close(self):
        if self._h:
            _cm.cm_shutdown(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- objects --
    def build_pieces(self, offsets, points) -> int:
        off = np.ascontiguousarray(offsets, np.int64)
        xyz = np.ascontiguousarray(points, np.float64)
        h = ctypes.c_uint32()
        self._check(_cm.cm_build_pieces(self._h, len(off) - 1, _ptr(off), _ptr(xyz), ctypes.byref(h)),
                    "cm_build_pieces")
        return h.value

    def build_raw(self, plane_off, planes, vert_off, verts, edge_off, edges) -> int:
        a = [np.ascontiguousarray(x, t) for x, t in ((plane_off, np.int64), (planes, np.float64),
                                                     (vert_off, np.int64), (verts, np.float64),
                                                     (edge_off, np.int64), (edges, np.int32))]
        h = ctypes.c_uint32()
        self._check(_cm.cm_build_pieces_raw(self._h, len(a[0]) - 1, *[_ptr(x) for x in a], ctypes.byref(h)),
                    "cm_build_pieces_raw")
        return h.value

    def build_objects(self, objects: Sequence) -> np.ndarray:
        """Registers generator objects (point clouds or explicit pieces); returns handles."""
        out = np.zeros(len(objects), np.uint32)
        pts_idx = [i for i, o in enumerate(objects) if hasattr(o, "points")]
        if pts_idx:
            obj_off, piece_off, xyz = [0], [0], []
            for i in pts_idx:
                o = objects[i]
                obj_off.append(obj_off[-1] + o.n_pieces)
                base = piece_off[-1]
                piece_off.extend((base + np.asarray(o.offsets[1:])).tolist())
                xyz.append(o.points)
            obj_off = np.array(obj_off, np.int64)
            piece_off = np.array(piece_off, np.int64)
            xyz = np.ascontiguousarray(np.concatenate(xyz), np.float64)
            hs = np.zeros(len(pts_idx), np.uint32)
            self._check(_cm.cm_build_objects(self._h, len(pts_idx), _ptr(obj_off), _ptr(piece_off), _ptr(xyz),
                                             _ptr(hs)), "cm_build_objects")
            out[pts_idx] = hs
        for i, o in enumerate(objects):
            if not hasattr(o, "points"):
                out[i] = self.build_raw(o.plane_off, o.planes, o.vert_off, o.verts, o.edge_off, o.edges)
        # primitive objects (contexts with sdf_kind = 2): their SDF side
        if self.params.sdf_kind == 2:
            for i, o in enumerate(objects):
                if getattr(o, "prim_rec", None) is not None:
                    self.object_set_prims(int(out[i]), o.prim_rec, o.prim_plane_off, o.prim_planes)
        return out

    def release(self, h: int):
        self._check(_cm.cm_release_object(self._h, int(h)), "cm_release_object")

    def object_info(self, h: int):
        k, p, v, e = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._check(_cm.cm_object_info(self._h, int(h), ctypes.byref(k), ctypes.byref(p), ctypes.byref(v),
                                       ctypes.byref(e)), "cm_object_info")
        return k.value, p.value, v.value, e.value

    def object_export(self, h: int) -> dict:
        K, P, V, E = self.object_info(h)
        po, vo, eo = np.zeros(K + 1, np.int64), np.zeros(K + 1, np.int64), np.zeros(K + 1, np.int64)
        pl, vs, es = np.zeros((P, 4)), np.zeros((V, 3)), np.zeros((E, 2), np.int32)
        self._check(_cm.cm_object_export(self._h, int(h), _ptr(po), _ptr(pl), _ptr(vo), _ptr(vs), _ptr(eo),
                                         _ptr(es)), "cm_object_export")
        return dict(plane_off=po, planes=pl, vert_off=vo, verts=vs, edge_off=eo, edges=es)

    def object_grid(self, h: int):
        meta = np.zeros(8, np.float32)
        self._check(_cm.cm_object_grid(self._h, int(h), None, _ptr(meta)), "cm_object_grid")
        n = int(meta[7])
        G = np.zeros(n ** 3, np.float32)
        self._check(_cm.cm_object_grid(self._h, int(h), _ptr(G), _ptr(meta)), "cm_object_grid")
        return G.reshape(n, n, n), meta[:3].astype(np.float64), meta[3:6].astype(np.float64), float(meta[6])

    def object_spline(self, h: int):
        """A spline object's (n, box origin [3], cell size [3], coefficients
        [4, n+3, n+3, n+3] of phi, n_x, n_y, n_z) (contexts with sdf_kind = 1)."""
        meta = np.zeros(7, np.float32)
        self._check(_cm.cm_object_spline(self._h, int(h), None, _ptr(meta)), "cm_object_spline")
        n = int(meta[0])
        C = np.zeros(((n + 3) ** 3, 4), np.float32)
        self._check(_cm.cm_object_spline(self._h, int(h), _ptr(C), _ptr(meta)), "cm_object_spline")
        return n, meta[1:4].astype(np.float64), meta[4:7].astype(np.float64), C.T.reshape(4, n + 3, n + 3, n + 3)

    def object_set_prims(self, h: int, rec, plane_off, planes):
        """The SDF side of object h as primitives (cm_object_set_prims; contexts
        with sdf_kind = 2): rec [n, 32] records, half-spaces planes [*, 4] indexed
        by plane_off [n + 1]."""
        rec = np.ascontiguousarray(rec, np.float64).reshape(-1, 32)
        off = np.ascontiguousarray(plane_off, np.int64)
        pl = np.ascontiguousarray(planes, np.float64).reshape(-1, 4)
        self._check(_cm.cm_object_set_prims(self._h, int(h), len(rec), _ptr(rec), _ptr(off), _ptr(pl)),
                    "cm_object_set_prims")

    def plan(self, qa, qb) -> "Plan":
        return Plan(self, qa, qb)


def make_queries(qa, qb, poses) -> np.ndarray:
    """Host cm_query array from object handles and [n, 14] poses (qa, ta, qb, tb)."""
    poses = np.asarray(poses, np.float64).reshape(-1, 14)
    q = np.zeros(len(poses), QUERY_DTYPE)
    q["a"] = np.asarray(qa, np.uint32)
    q["b"] = np.asarray(qb, np.uint32)
    q["qa"] = poses[:, 0:4]
    q["ta"] = poses[:, 4:7]
    q["qb"] = poses[:, 7:11]
    q["tb"] = poses[:, 11:14]
    return q


def groups_struct(t) -> cm_groups:
    """cm_groups pointing into the rows of a [12, G] float32 device tensor."""
    G = t.shape[1]
    base = t.data_ptr()
    rows = lambda r: ctypes.c_void_p(base + 4 * r * G)
    return cm_groups(rows(0), rows(3), rows(6), rows(7), rows(10), rows(11))


class Plan:
    """Fixed objects of a batch of pair-queries plus the launch scratch."""

    def __init__(self, ctx: Context, qa, qb):
        self.ctx = ctx
        self.qa = np.asarray(qa, np.uint32)
        self.qb = np.asarray(qb, np.uint32)
        hq = make_queries(self.qa, self.qb, np.tile([1, 0, 0, 0, 0, 0, 0] * 2, (len(self.qa), 1)))
        self._h = ctypes.c_void_p()
        ctx._check(_cm.cm_plan_create(ctx.handle, _ptr(hq), len(hq), ctypes.byref(self._h)), "cm_plan_create")
        self._info()

    @classmethod
    def reserve(cls, ctx: Context, max_queries: int, max_groups: int, max_contacts: int) -> "Plan":
        """A plan of fixed capacity holding an empty batch (cm_plan_reserve);
        refill() replaces its batch.  Records and cotangents are [12, max_groups],
        gradients and directions [max_queries, 12]; the first G (n) rows are the
        batch's."""
        self = cls.__new__(cls)
        self.ctx = ctx
        self.qa = np.zeros(0, np.uint32)
        self.qb = np.zeros(0, np.uint32)
        self._h = ctypes.c_void_p()
        ctx._check(_cm.cm_plan_reserve(ctx.handle, int(max_queries), int(max_groups), int(max_contacts),
                                       ctypes.byref(self._h)), "cm_plan_reserve")
        self._info()
        return self

    def refill(self, qa, qb, stream=None):
        """Replace the batch of a reserved plan (cm_plan_refill, enqueued on `stream`)."""
        qa = np.asarray(qa, np.uint32)
        qb = np.asarray(qb, np.uint32)
        hq = make_queries(qa, qb, np.tile([1, 0, 0, 0, 0, 0, 0] * 2, (len(qa), 1)))
        self.ctx._check(_cm.cm_plan_refill(self.ctx.handle, self._h, _ptr(hq), len(hq), _stream_ptr(stream)),
                        "cm_plan_refill")
        self.qa, self.qb = qa, qb
        self._info()

    def _info(self):
        G, C, n = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _cm.cm_plan_info(self._h, ctypes.byref(G), ctypes.byref(C), ctypes.byref(n))
        self.G, self.C, self.n = G.value, C.value, n.value
        self.group_off = np.zeros(self.n + 1, np.int64)
        self.contact_off = np.zeros(self.n + 1, np.int64)
        _cm.cm_plan_offsets(self._h, _ptr(self.group_off), _ptr(self.contact_off))
        mq, mg, mc = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        _cm.cm_plan_capacity(self._h, ctypes.byref(mq), ctypes.byref(mg), ctypes.byref(mc))
        # rows of the record (group) and per-query arrays the kernels address:
        # the capacity of a reserved plan, else the batch's own sizes
        self.rows_G, self.rows_n, self.cap_C = mg.value, mq.value, mc.value

    @property
    def handle(self):
        return self._h

    def destroy(self):
        if self._h:
            _cm.cm_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def device_queries(self, poses, device="cuda"):
        """Device cm_query array (torch uint8 [n, 64]) for this plan's objects."""
        torch = _torch()
        hq = make_queries(self.qa, self.qb, poses)
        return torch.from_numpy(hq.view(np.uint8).reshape(-1, 64).copy()).to(device)

    def write_queries(self, q_buf, poses):
        """Write the batch's device queries into the first n rows of q_buf
        (torch uint8 [rows, 64], rows >= n: e.g. a reserved plan's rows_n, the
        buffer a graph was captured with)."""
        torch = _torch()
        hq = make_queries(self.qa, self.qb, poses)
        q_buf[: self.n].copy_(torch.from_numpy(hq.view(np.uint8).reshape(-1, 64).copy()))
        return q_buf

    def forward(self, q_dev, out=None, debug: bool = False, stream=None):
        """Group records [12, G] (rows p, n, d, q, W, logZ) and optional per-contact [13, C]."""
        torch = _torch()
        if out is None:
            out = torch.empty((12, self.rows_G), dtype=torch.float32, device=q_dev.device)
        dbg = torch.empty((13, self.C), dtype=torch.float32, device=q_dev.device) if debug else None
        st = _cm.cm_contacts_fwd(self.ctx.handle, self._h, ctypes.c_void_p(q_dev.data_ptr()), groups_struct(out),
                                 ctypes.c_void_p(dbg.data_ptr()) if dbg is not None else None,
                                 _stream_ptr(stream))
        self.ctx._check(st, "cm_contacts_fwd")
        return (out, dbg) if debug else out

    def project(self, q_dev, points, out=None, stream=None):
        """Isosurface projection (cm_project_points) of one point per group,
        points [3, G] (world; e.g. the records' first three rows)."""
        torch = _torch()
        pin = points.contiguous()
        if out is None:
            out = torch.empty_like(pin)
        st = _cm.cm_project_points(self.ctx.handle, self._h, ctypes.c_void_p(q_dev.data_ptr()),
                                   ctypes.c_void_p(pin.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   _stream_ptr(stream))
        self.ctx._check(st, "cm_project_points")
        return out

    def forward_noalloc(self, q_dev, out, stream=None):
        """The forward records into the caller's `out` [12, G] with the launch
        scratch in the library's fixed device array (cm_contacts_fwd_noalloc):
        nothing is allocated by this call."""
        st = _cm.cm_contacts_fwd_noalloc(self.ctx.handle, self._h, ctypes.c_void_p(q_dev.data_ptr()),
                                         groups_struct(out), _stream_ptr(stream))
        self.ctx._check(st, "cm_contacts_fwd_noalloc")
        return out

    def backward(self, q_dev, cot, grad=None, stream=None):
        torch = _torch()
        if grad is None:
            grad = torch.empty((self.rows_n, 12), dtype=torch.float32, device=q_dev.device)
        st = _cm.cm_contacts_bwd(self.ctx.handle, self._h, ctypes.c_void_p(q_dev.data_ptr()), groups_struct(cot),
                                 ctypes.c_void_p(grad.data_ptr()), _stream_ptr(stream))
        self.ctx._check(st, "cm_contacts_bwd")
        return grad

    def step(self, q_dev, cot, direction=None, out=None, grad=None, hv=None, records=True, stream=None):
        """Records [12, G] (if records), gradient [n, 12] and, with a direction, H v [n, 12]
        from one forward sweep and one adjoint (cm_contacts_step)."""
        torch = _torch()
        if records and out is None:
            out = torch.empty((12, self.rows_G), dtype=torch.float32, device=q_dev.device)
        if grad is None:
            grad = torch.empty((self.rows_n, 12), dtype=torch.float32, device=q_dev.device)
        if direction is not None and hv is None:
            hv = torch.empty((self.rows_n, 12), dtype=torch.float32, device=q_dev.device)
        st = _cm.cm_contacts_step(self.ctx.handle, self._h, ctypes.c_void_p(q_dev.data_ptr()),
                                  groups_struct(out) if records else _cm.cm_groups(), groups_struct(cot),
                                  ctypes.c_void_p(grad.data_ptr()),
                                  ctypes.c_void_p(direction.data_ptr()) if direction is not None else None,
                                  ctypes.c_void_p(hv.data_ptr()) if direction is not None else None,
                                  _stream_ptr(stream))
        self.ctx._check(st, "cm_contacts_step")
        return (out if records else None), grad, (hv if direction is not None else None)

    def graph(self, q_dev, cot, grad, direction=None, hv=None, out=None) -> "Graph":
        """HIP graph of step() with these device buffers (cm_graph_create)."""
        h = ctypes.c_void_p()
        st = _cm.cm_graph_create(self.ctx.handle, self._h, ctypes.c_void_p(q_dev.data_ptr()),
                                 groups_struct(out) if out is not None else _cm.cm_groups(), groups_struct(cot),
                                 ctypes.c_void_p(grad.data_ptr()),
                                 ctypes.c_void_p(direction.data_ptr()) if direction is not None else None,
                                 ctypes.c_void_p(hv.data_ptr()) if hv is not None else None, ctypes.byref(h))
        self.ctx._check(st, "cm_graph_create")
        return Graph(self, h, (q_dev, cot, grad, direction, hv, out))

    def autotune(self, q_dev, cot, grad, direction=None, hv=None, stream=None) -> int:
        """Picks the persistent launch shape for this plan (cm_plan_autotune); returns workgroups per CU."""
        best = ctypes.c_int32()
        st = _cm.cm_plan_autotune(self.ctx.handle, self._h, ctypes.c_void_p(q_dev.data_ptr()), groups_struct(cot),
                                  ctypes.c_void_p(grad.data_ptr()),
                                  ctypes.c_void_p(direction.data_ptr()) if direction is not None else None,
                                  ctypes.c_void_p(hv.data_ptr()) if hv is not None else None,
                                  _stream_ptr(stream), ctypes.byref(best))
        self.ctx._check(st, "cm_plan_autotune")
        return int(best.value)

    @property
    def launch_shape(self) -> tuple:
        """(float sweeps, dual sweeps) persistent workgroups per CU."""
        f, d = ctypes.c_int32(), ctypes.c_int32()
        self.ctx._check(_cm.cm_plan_launch_shape(self._h, ctypes.byref(f), ctypes.byref(d)), "cm_plan_launch_shape")
        return int(f.value), int(d.value)

    @launch_shape.setter
    def launch_shape(self, shape):
        self.ctx._check(_cm.cm_plan_set_launch_shape(self._h, int(shape[0]), int(shape[1])),
                        "cm_plan_set_launch_shape")

    @property
    def wg_waves(self) -> tuple:
        """(float sweeps, dual sweeps) waves per workgroup of the narrow phase."""
        f, d = ctypes.c_int32(), ctypes.c_int32()
        self.ctx._check(_cm.cm_plan_wg_waves(self._h, ctypes.byref(f), ctypes.byref(d)), "cm_plan_wg_waves")
        return int(f.value), int(d.value)

    @wg_waves.setter
    def wg_waves(self, waves):
        self.ctx._check(_cm.cm_plan_set_wg_waves(self._h, int(waves[0]), int(waves[1])), "cm_plan_set_wg_waves")

    def hvp(self, q_dev, cot, direction, hv=None, grad=None, stream=None):
        torch = _torch()
        if hv is None:
            hv = torch.empty((self.rows_n, 12), dtype=torch.float32, device=q_dev.device)
        st = _cm.cm_hvp(self.ctx.handle, self._h, ctypes.c_void_p(q_dev.data_ptr()), groups_struct(cot),
                        ctypes.c_void_p(direction.data_ptr()), ctypes.c_void_p(hv.data_ptr()),
                        ctypes.c_void_p(grad.data_ptr()) if grad is not None else None, _stream_ptr(stream))
        self.ctx._check(st, "cm_hvp")
        return hv

    def jvp(self, q_dev, direction, out=None, out_t=None, stream=None):
        """Records [12, G] and their derivatives along `direction` [n, 12]
        (cm_contacts_jvp)."""
        torch = _torch()
        if out is None:
            out = torch.empty((12, self.rows_G), dtype=torch.float32, device=q_dev.device)
        if out_t is None:
            out_t = torch.empty((12, self.rows_G), dtype=torch.float32, device=q_dev.device)
        st = _cm.cm_contacts_jvp(self.ctx.handle, self._h, ctypes.c_void_p(q_dev.data_ptr()), groups_struct(out),
                                 groups_struct(out_t), ctypes.c_void_p(direction.data_ptr()), _stream_ptr(stream))
        self.ctx._check(st, "cm_contacts_jvp")
        return out, out_t

    def set_timing(self, enable: bool = True):
        self.ctx._check(_cm.cm_plan_set_timing(self._h, int(enable)), "cm_plan_set_timing")

    def timing(self) -> dict:
        """Last kernel durations (ms) measured with HIP events on the launch stream."""
        ms = np.zeros(5, np.float32)
        self.ctx._check(_cm.cm_plan_timing(self._h, _ptr(ms)), "cm_plan_timing")
        return dict(broad=float(ms[0]), narrow_fwd=float(ms[1]), narrow_tan=float(ms[2]),
                    narrow_adj=float(ms[3]), narrow_dual_adj=float(ms[4]))

    def work(self) -> tuple:
        """Point-plane evaluations performed by the last pass for vertex and for
        edge contacts (cm_plan_work)."""
        v = np.zeros(2, np.int64)
        self.ctx._check(_cm.cm_plan_work(self._h, _ptr(v)), "cm_plan_work")
        return int(v[0]), int(v[1])

    def stats(self) -> dict:
        s = np.zeros(8, np.int64)
        self.ctx._check(_cm.cm_plan_stats(self._h, _ptr(s)), "cm_plan_stats")
        return dict(surv_verts=int(s[0]), surv_edges=int(s[1]), tiles=int(s[2]), verts=int(s[3]),
                    edges=int(s[4]), pairs=int(s[5]), vertex_pairs=int(s[6]), edge_pairs=int(s[7]))


class Graph:
    """A captured step (cm_graph_*); keeps its plan and buffers alive."""

    def __init__(self, plan, h, keep):
        self.plan, self._h, self._keep = plan, h, keep

    def launch(self, stream=None):
        self.plan.ctx._check(_cm.cm_graph_launch(self._h, _stream_ptr(stream)), "cm_graph_launch")

    def __del__(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _cm.cm_graph_destroy(self._h)
            self._h = None


class Server:
    """Client side of the serving loop (cm_submit / cm_poll / cm_wait).

    Requests are host arrays; their results are written into host buffers
    owned by the returned Ticket and are valid once it is done.
    """

    def __init__(self, ctx: Context):
        self.ctx = ctx
        self._npieces = {}

    def _pieces(self, h: int) -> int:
        k = self._npieces.get(h)
        if k is None:
            k = self._npieces[h] = self.ctx.object_info(h)[0]
        return k

    def submit(self, qa, qb, poses, cotangent=None) -> "Ticket":
        q = make_queries(qa, qb, poses)
        G = int(sum(self._pieces(int(a)) + self._pieces(int(b)) for a, b in zip(qa, qb)))
        out = np.zeros((G, 12), np.float32)
        grad = np.zeros((len(q), 12), np.float32) if cotangent is not None else None
        cot = np.ascontiguousarray(cotangent, np.float32).reshape(G, 12) if cotangent is not None else None
        req = _cm.cm_request(q=_ptr(q), n=len(q), want_grad=int(cotangent is not None),
                             cotangent=_ptr(cot) if cot is not None else None, out_groups=_ptr(out),
                             out_grad=_ptr(grad) if grad is not None else None)
        t = ctypes.c_uint64()
        self.ctx._check(_cm.cm_submit(self.ctx.handle, ctypes.byref(req), ctypes.byref(t)), "cm_submit")
        return Ticket(self, t.value, q, cot, out, grad)

    def latencies(self) -> np.ndarray:
        """Seconds from submit to results written, of requests completed since the last call."""
        out = []
        while True:
            buf = np.zeros(65536)
            n = ctypes.c_int64()
            self.ctx._check(_cm.cm_serve_latencies(self.ctx.handle, _ptr(buf), len(buf), ctypes.byref(n)),
                            "cm_serve_latencies")
            out.append(buf[:n.value])
            if n.value < len(buf):
                return np.concatenate(out)

    def stats(self) -> dict:
        s = np.zeros(7, np.int64)
        self.ctx._check(_cm.cm_serve_stats(self.ctx.handle, _ptr(s)), "cm_serve_stats")
        return dict(submitted=int(s[0]), completed=int(s[1]), batches=int(s[2]), queued=int(s[3]),
                    in_flight=int(s[4]), peak_device_bytes=int(s[5]), queries=int(s[6]))


class Ticket:
    def __init__(self, server, tid, q, cot, out, grad):
        self.server, self.id = server, tid
        self._keep = (q, cot)  # inputs are copied at submit; kept for symmetry
        self.out, self.grad = out, grad
        self.status = None

    def poll(self) -> bool:
        if self.status is not None:
            return True
        done, res = ctypes.c_int32(), ctypes.c_int32()
        self.server.ctx._check(_cm.cm_poll(self.server.ctx.handle, self.id, ctypes.byref(done), ctypes.byref(res)),
                               "cm_poll")
        if done.value:
            self.status = res.value
        return bool(done.value)

    def wait(self, timeout_ms: int = 60000):
        if self.status is None:
            res = ctypes.c_int32()
            self.server.ctx._check(_cm.cm_wait(self.server.ctx.handle, self.id, int(timeout_ms), ctypes.byref(res)),
                                   "cm_wait")
            self.status = res.value
        if self.status != 0:
            raise CMError(self.status, "request failed")
        return self.out, self.grad


# ------------------------------------------------------------------ autograd --
def _require_zero(xi):
    if bool(xi.detach().any()):
        raise ValueError("ContactFn evaluates the records at the plan's poses, i.e. at xi = 0; retract a "
                         "perturbation into the poses (R <- exp([w]x) R, t <- t + v) and write new queries instead")


def _torch_fn():
    torch = _torch()

    class HvpFn(torch.autograd.Function):
        """u -> H_c u, the Hessian of L = <c, y> w.r.t. xi along u (cm_hvp).
        Linear in u with H symmetric, so its backward along w is H_c w.  Third
        derivatives (w.r.t. xi or c) are not provided."""

        @staticmethod
        def forward(ctx, u, xi, cot, plan, q_dev):
            ctx.plan, ctx.q_dev = plan, q_dev
            ctx.save_for_backward(cot)
            return plan.hvp(q_dev, cot, u.detach().contiguous())

        @staticmethod
        def backward(ctx, w):
            (cot,) = ctx.saved_tensors
            gu = HvpFn.apply(w.contiguous(), None, cot, ctx.plan, ctx.q_dev) if ctx.needs_input_grad[0] else None
            return gu, None, None, None, None

    class JvpFn(torch.autograd.Function):
        """u -> J u, the derivative of the records along the pose direction u
        (cm_contacts_jvp).  Its backward along w: J^T w (cm_contacts_bwd) for u,
        and H_w u (cm_hvp with cotangent w) for xi."""

        @staticmethod
        def forward(ctx, u, xi, plan, q_dev):
            ctx.plan, ctx.q_dev = plan, q_dev
            u = u.detach().contiguous()
            ctx.save_for_backward(u, xi)
            return plan.jvp(q_dev, u)[1]

        @staticmethod
        def backward(ctx, w):
            u, xi = ctx.saved_tensors
            w = w.contiguous()
            gu = ContactGrad.apply(xi, w, ctx.plan, ctx.q_dev) if ctx.needs_input_grad[0] else None
            gx = HvpFn.apply(u, xi, w, ctx.plan, ctx.q_dev) if ctx.needs_input_grad[1] else None
            return gu, gx, None, None

    class ContactGrad(torch.autograd.Function):
        """(xi, c) -> dL/dxi for L = <c, y(xi)> (cm_contacts_bwd).  Its backward
        along v: H_c v w.r.t. xi (cm_hvp) and J v w.r.t. c (cm_contacts_jvp), each
        itself differentiable in v, so torch.autograd.functional.hvp's
        double-backward works."""

        @staticmethod
        def forward(ctx, xi, cot, plan, q_dev):
            ctx.plan, ctx.q_dev = plan, q_dev
            cot = cot.detach().contiguous()
            ctx.save_for_backward(xi, cot)
            return plan.backward(q_dev, cot)

        @staticmethod
        def backward(ctx, v):
            xi, cot = ctx.saved_tensors
            v = v.contiguous()
            gx = HvpFn.apply(v, xi, cot, ctx.plan, ctx.q_dev) if ctx.needs_input_grad[0] else None
            gc = JvpFn.apply(v, xi, ctx.plan, ctx.q_dev) if ctx.needs_input_grad[1] else None
            return gx, gc, None, None

    class ContactFn(torch.autograd.Function):
        """Group records y [12, G] (rows p, n, d, q, W, logZ) of a plan's batch as
        a function of the pose perturbation xi [n, 12] = (w_A, v_A, w_B, v_B) per
        query, T_X <- (exp([w_X]x) R_X, t_X + v_X), evaluated at xi = 0 (the
        poses in q_dev; a nonzero xi is rejected).  forward: cm_contacts_fwd;
        backward: cm_contacts_bwd, through ContactGrad, whose own backward calls
        cm_hvp and cm_contacts_jvp, so torch.autograd.grad and
        torch.autograd.functional.hvp over xi work for any loss of the records.
        The derivatives are those of the pose twist at zero (the ones the
        adjoint kernels compute); use: ContactFn.apply(xi, plan, q_dev)."""

        @staticmethod
        def forward(ctx, xi, plan, q_dev):
            _require_zero(xi)
            ctx.plan, ctx.q_dev = plan, q_dev
            ctx.save_for_backward(xi)
            return plan.forward(q_dev)

        @staticmethod
        def backward(ctx, gy):
            (xi,) = ctx.saved_tensors
            return ContactGrad.apply(xi, gy.contiguous(), ctx.plan, ctx.q_dev), None, None

    return ContactFn, ContactGrad, HvpFn, JvpFn


_FNS = None


def __getattr__(name):
    # the autograd classes are created on first use, so that importing this
    # module does not import torch
    global _FNS
    if name in ("ContactFn", "ContactGrad", "HvpFn", "JvpFn"):
        if _FNS is None:
            _FNS = dict(zip(("ContactFn", "ContactGrad", "HvpFn", "JvpFn"), _torch_fn()))
        return _FNS[name]
    raise AttributeError(name)
