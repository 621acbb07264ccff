"""Pins of the oracle's primitive-based SDFs (Sec. III-A): the superquadric's
radial SDF, the PSQ, the XPSQ's projection onto its quadratic spline (soft
Cardano branches) and its swept SDF, and the CSG fold -- against closed forms,
the superquadric's parametric surface, its homogeneity along rays, and brute
force over the spline parameter."""
import numpy as np
import pytest

import oracle as O

pytestmark = []


def _rec(kind, op=0, c=(0, 0, 0), p=None, quat=(1, 0, 0, 0), a0=(1, 1, 1), e0=(1, 1), a1=None, e1=None):
    r = np.zeros(32)
    r[0], r[1] = kind, op
    if p is None:
        r[2:5] = c
    else:
        r[2:11] = np.asarray(p, float).ravel()
    r[11:15] = quat
    r[15:18], r[18:20] = a0, e0
    r[20:23] = a0 if a1 is None else a1
    r[23:25] = e0 if e1 is None else e1
    return r


def _obj(recs, planes_per=None):
    """An oracle object with one small tetrahedron piece (the mesh side, unused
    here) and the given primitives as its SDF side."""
    t = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float) * 0.01
    o = O.from_points(np.array([0, 4]), t)
    planes_per = planes_per or [np.zeros((0, 4))] * len(recs)
    off = np.concatenate([[0], np.cumsum([len(p) for p in planes_per])]).astype(np.int64)
    o.set_prims(np.array(recs), off, np.concatenate(planes_per) if off[-1] else np.zeros((0, 4)))
    return o


def _sq_surface(a, e, n=400, seed=0):
    """Points of the superquadric f = 1 from its parametric form
    x = a_x C(eta)^e1 C(om)^e2, y = a_y C(eta)^e1 S(om)^e2, z = a_z S(eta)^e1,
    C(u)^k = sign(cos u) |cos u|^k (S likewise)."""
    rng = np.random.default_rng(seed)
    eta = rng.uniform(-np.pi / 2, np.pi / 2, n)
    om = rng.uniform(-np.pi, np.pi, n)
    sp = lambda v, k: np.sign(v) * np.abs(v) ** k
    return np.stack([a[0] * sp(np.cos(eta), e[0]) * sp(np.cos(om), e[1]),
                     a[1] * sp(np.cos(eta), e[0]) * sp(np.sin(om), e[1]),
                     a[2] * sp(np.sin(eta), e[0])], 1)


def test_sphere_is_exact():
    prm = O.default_params(0.1)
    o = _obj([_rec(0, c=(0.1, -0.2, 0.05), a0=(0.3, 0.3, 0.3), e0=(1, 1))])
    rng = np.random.default_rng(1)
    x = rng.normal(size=(200, 3)) * 0.4 + [0.1, -0.2, 0.05]
    phi, g = o.prims_eval(prm, x)
    r = np.linalg.norm(x - [0.1, -0.2, 0.05], axis=1)
    keep = r > 0.03
    # the regulariser (q^2 + delta^2, delta = 1e-3) moves f by 3 delta^2 and the
    # radius by delta^2 R^2 / (2 |x|): |phi - (|x| - R)| <= 2 delta^2 (R^3/|x|^2 + R^2/|x|)
    d2, R = 1e-6, 0.3
    bound = 2 * d2 * (R ** 3 / r ** 2 + R ** 2 / r)
    assert (np.abs(phi - (r - 0.3))[keep] <= bound[keep]).all()
    u = (x - [0.1, -0.2, 0.05]) / r[:, None]
    assert np.allclose(g[keep], u[keep], atol=1e-4)


@pytest.mark.parametrize("a,e", [((0.3, 0.2, 0.1), (1.0, 1.0)), ((0.2, 0.3, 0.25), (0.3, 0.8)),
                                 ((0.25, 0.15, 0.3), (1.6, 0.5))])
def test_superquadric_surface_and_rays(a, e):
    """phi = 0 on the parametric surface f = 1, and along the ray through a
    surface point s, phi(lambda s) = (lambda - 1) |s| (f is homogeneous of
    degree 2/e1 along rays, so f(lambda s)^(-e1/2) = 1/lambda)."""
    prm = O.default_params(0.1)
    o = _obj([_rec(0, a0=a, e0=e)])
    s = _sq_surface(a, e)
    # the regulariser (q^2 + delta^2) changes f by a relative amount of at most
    # 2 max(1/e1, 1/e2) delta^2 / min_k q_k^2, hence phi by |x| e1 / 2 times that
    sc = s / np.array(a)
    keep = (np.abs(sc) > 0.05).all(1)
    s, sc = s[keep], sc[keep]
    rel = 2 * max(1 / e[0], 1 / e[1]) * 1e-6 / (sc ** 2).min(1)
    r = np.linalg.norm(s, axis=1)
    phi, _ = o.prims_eval(prm, s)
    assert (np.abs(phi) <= r * e[0] * rel + 1e-12).all()
    for lam in (0.5, 1.7):
        p2, _ = o.prims_eval(prm, lam * s)
        assert (np.abs(p2 - (lam - 1) * r) <= lam * r * e[0] * rel / min(lam, 1) ** 2 + 1e-12).all()


def test_rotation_and_planes():
    """A PSQ turned by a quaternion equals the unturned one at the counter-turned
    point; with a half-space its SDF lies within [max, max + tau log 2] of the
    SQ's and the plane's."""
    prm = O.default_params(0.1)
    th = 0.7
    q = (np.cos(th / 2), 0.0, 0.0, np.sin(th / 2))  # about z
    R = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    c = np.array([0.05, 0.02, -0.01])
    pl = np.array([[0.0, 1.0, 0.0, -0.05]])  # y <= 0.05 in the PSQ frame
    o = _obj([_rec(0, c=c, quat=q, a0=(0.3, 0.2, 0.1), e0=(0.5, 0.7))], [pl])
    o0 = _obj([_rec(0, a0=(0.3, 0.2, 0.1), e0=(0.5, 0.7))])
    rng = np.random.default_rng(2)
    xl = rng.uniform(-0.4, 0.4, (300, 3))
    x = xl @ R.T + c
    phi, _ = o.prims_eval(prm, x)
    sq, _ = o0.prims_eval(prm, xl)
    plane = xl[:, 1] - 0.05
    m = np.maximum(sq, plane)
    assert (phi >= m - 1e-12).all() and (phi <= m + prm.tau_cap * np.log(2) + 1e-12).all()


def _bezier(P, t):
    t = np.asarray(t)[..., None]
    return (1 - t) ** 2 * P[0] + 2 * t * (1 - t) * P[1] + t ** 2 * P[2]


SPINE = np.array([[0.0, 0.0, 0.0], [0.3, 0.4, 0.05], [0.6, 0.0, 0.1]])


def test_projection_roots_contain_the_closest_point():
    """With sharp temperatures, one of the three t* is the parameter of the
    spline point closest to x (brute force over t in [0, 1]), interior or at an
    end."""
    prm = O.default_params(0.1, tau_t=1e-7, tau_disc=1e-9)
    o = _obj([_rec(1, p=SPINE, a0=(0.05, 0.05, 0.05))])
    rng = np.random.default_rng(3)
    x = rng.uniform([-0.3, -0.3, -0.2], [0.9, 0.7, 0.3], (400, 3))
    t = o.xpsq_roots(prm, 0, x)
    tg = np.linspace(0, 1, 200001)
    curve = _bezier(SPINE, tg)
    for i in range(len(x)):
        d = np.linalg.norm(curve - x[i], axis=1)
        dmin = d.min()
        dr = np.linalg.norm(_bezier(SPINE, t[i]) - x[i], axis=1).min()
        assert dr <= dmin + 1e-7, (i, x[i], t[i], tg[np.argmin(d)])


def test_swept_sphere_is_a_tube():
    """A sphere of radius r swept along the spline: with sharp temperatures the
    XPSQ SDF is the distance to the spline minus r."""
    prm = O.default_params(0.1, tau_t=1e-7, tau_disc=1e-9, tau_cup=1e-7, tau_cap=1e-7)
    r = 0.06
    o = _obj([_rec(1, p=SPINE, a0=(r, r, r), e0=(1, 1))])
    rng = np.random.default_rng(4)
    x = rng.uniform([-0.3, -0.3, -0.2], [0.9, 0.7, 0.3], (300, 3))
    phi, _ = o.prims_eval(prm, x)
    curve = _bezier(SPINE, np.linspace(0, 1, 200001))
    dist = np.array([np.linalg.norm(curve - xi, axis=1).min() for xi in x])
    keep = dist > 0.01
    assert np.allclose(phi[keep], dist[keep] - r, atol=5e-6)


def test_roots_match_the_cubic():
    """With sharp temperatures the three t* are the real roots of the
    stationarity cubic 2|A|^2 t^3 + 3 A.B t^2 + (|B|^2 + 2 A.(p1 - x)) t + B.(p1 - x)
    (numpy's companion-matrix roots), clipped to [0, 1]: the single real root
    three times, or the three roots, as Cardano's branches give them; at the
    default temperatures every t* lies in [0, 1]."""
    sharp = O.default_params(0.1, tau_t=1e-9, tau_disc=1e-12)
    o = _obj([_rec(1, p=SPINE, a0=(0.05, 0.05, 0.05))])
    A = SPINE[0] - 2 * SPINE[1] + SPINE[2]
    B = 2 * (SPINE[1] - SPINE[0])
    rng = np.random.default_rng(5)
    x = rng.uniform([-1.0, -1.0, -0.5], [1.6, 1.5, 0.6], (400, 3))
    t = o.xpsq_roots(sharp, 0, x)
    n_one = n_three = 0
    for i in range(len(x)):
        C0 = SPINE[0] - x[i]
        rts = np.roots([2 * A @ A, 3 * A @ B, B @ B + 2 * A @ C0, B @ C0])
        real = np.sort(rts[np.abs(rts.imag) < 1e-7].real)
        if len(real) == 1:
            n_one += 1
            assert np.allclose(t[i], np.clip(real[0], 0, 1), atol=1e-6), (i, t[i], real)
        elif len(real) == 3 and np.diff(real).min() > 1e-3:
            n_three += 1
            assert np.allclose(np.sort(t[i]), np.clip(real, 0, 1), atol=1e-6), (i, t[i], real)
    assert n_one > 50 and n_three > 50
    td = o.xpsq_roots(O.default_params(0.1), 0, x)
    assert (td >= -1e-12).all() and (td <= 1 + 1e-12).all()


def test_csg_fold():
    """Union, subtraction and intersection of two spheres against the smooth
    min / max of their exact SDFs."""
    prm = O.default_params(0.1)
    c1, c2, r1, r2 = np.array([0.0, 0, 0]), np.array([0.15, 0, 0]), 0.2, 0.12
    rng = np.random.default_rng(6)
    x = rng.uniform(-0.4, 0.4, (200, 3))
    d1 = np.linalg.norm(x - c1, axis=1) - r1
    d2 = np.linalg.norm(x - c2, axis=1) - r2
    n1, n2 = np.linalg.norm(x - c1, axis=1), np.linalg.norm(x - c2, axis=1)
    keep = (n1 > 0.03) & (n2 > 0.03)
    # each sphere within its regulariser bound (test_sphere_is_exact); smooth
    # min / max are 1-Lipschitz in each argument
    bnd = lambda R, r: 2e-6 * (R ** 3 / r ** 2 + R ** 2 / r)
    bound = np.maximum(bnd(r1, n1), bnd(r2, n2))
    lse = lambda a, b, tau: np.logaddexp(a / tau, b / tau) * tau
    for op, ref in ((0, -lse(-d1, -d2, prm.tau_cup)), (1, lse(d1, -d2, prm.tau_cap)), (2, lse(d1, d2, prm.tau_cap))):
        o = _obj([_rec(0, c=c1, a0=(r1,) * 3), _rec(0, op=op, c=c2, a0=(r2,) * 3)])
        phi, _ = o.prims_eval(prm, x)
        assert (np.abs(phi - ref)[keep] <= bound[keep] + 1e-12).all(), op


def test_gradient_matches_central_differences():
    prm = O.default_params(0.1)
    pl = np.array([[0.0, 0.0, 1.0, -0.02]])
    o = _obj([_rec(1, p=SPINE, a0=(0.06, 0.04, 0.05), e0=(0.6, 0.9), a1=(0.04, 0.05, 0.05), e1=(0.9, 0.5)),
              _rec(0, op=1, c=(0.3, 0.1, 0.0), a0=(0.05, 0.05, 0.05))], [pl, np.zeros((0, 4))])
    rng = np.random.default_rng(7)
    x = rng.uniform([-0.1, -0.1, -0.1], [0.7, 0.4, 0.2], (100, 3))
    phi, g = o.prims_eval(prm, x)
    h = 1e-6
    fd = np.zeros_like(g)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd[:, k] = (o.prims_eval(prm, x + e)[0] - o.prims_eval(prm, x - e)[0]) / (2 * h)
    assert np.allclose(g, fd, atol=1e-5 * (1 + np.abs(g)))


def test_sweep_frame_orientation():
    """The PSQ's axes along the spline: x along the in-plane normal N = b x T,
    y along the binormal b (B x A), z along the tangent T.  An ellipsoid with
    three different scales swept along the spline: from p(t0), along N the SDF
    is s - a_x, along b it is s - a_y (the point projects back to t0; on an
    axis the radial distance is exact)."""
    prm = O.default_params(0.1, tau_t=1e-7, tau_disc=1e-9, tau_cup=1e-7)
    a = (0.05, 0.03, 0.02)
    o = _obj([_rec(1, p=SPINE, a0=a, e0=(1, 1))])
    A = SPINE[0] - 2 * SPINE[1] + SPINE[2]
    B = 2 * (SPINE[1] - SPINE[0])
    b = np.cross(B, A)
    b /= np.linalg.norm(b)
    for t0 in (0.3, 0.55):
        T = 2 * A * t0 + B
        T /= np.linalg.norm(T)
        N = np.cross(b, T)
        p0 = _bezier(SPINE, t0)
        s = np.array([0.01, 0.03, 0.045, 0.07])
        phiN, _ = o.prims_eval(prm, p0 + s[:, None] * N)
        phib, _ = o.prims_eval(prm, p0 + s[:, None] * b)
        assert np.allclose(phiN, s - a[0], atol=2e-5), (t0, phiN, s - a[0])
        assert np.allclose(phib, s - a[1], atol=2e-5), (t0, phib, s - a[1])
