"""Pins of the oracle's projected-Jacobi step (Alg. 1, Eqs. (1)-(5), Sec. II-A).

Each test checks the oracle against something the mathematics fixes:
closed-form collisions, a block sliding on a plane, an incline at the
friction angle, free fall, momentum conservation, the friction cone, order
independence, and the frictionless LCP solved by active-set enumeration."""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from paper_2306_01369_amd import scenes

RHO = 2500.0


def mass(r):
    return RHO * 4.0 / 3.0 * math.pi * r ** 3


def _two(x0, x1, v0, v1, r=0.5, **kw):
    x = np.array([x0, x1], np.float64)
    v = np.array([v0, v1], np.float64)
    kw.setdefault("gravity", (0.0, 0.0, 0.0))
    return O.Oracle(x, v, np.array([r, r], np.float32), **kw)


def test_head_on_equal_spheres_reach_centre_of_mass_velocity():
    # touching (psi = 0), approaching at 1 m/s each: perfectly inelastic, both
    # end at v_cm = 0 after iteration 1, which is then a fixed point.
    for iters in (1, 2, 20):
        o = _two([0, 0, 0], [1, 0, 0], [1, 0, 0], [-1, 0, 0], n_iters=iters, mu=0.5)
        d = o.step(detail=True)
        assert d["n_pp"] == 1
        np.testing.assert_allclose(o.v, 0.0, atol=1e-14)
        m = mass(0.5)
        # impulse on particle 0 (first member) is -m*1 along x
        np.testing.assert_allclose(d["impulses"][0], [-m, 0, 0], rtol=1e-14)


def test_unequal_masses_inelastic_closed_form():
    x = np.array([[0, 0, 0], [1.5, 0, 0]], np.float64)      # r = 0.5 and 1.0: touching
    v = np.array([[2.0, 0, 0], [0.0, 0, 0]])
    r = np.array([0.5, 1.0], np.float32)
    o = O.Oracle(x, v, r, gravity=(0, 0, 0), n_iters=5)
    o.step()
    m0, m1 = mass(0.5), mass(1.0)
    vcm = (m0 * 2.0) / (m0 + m1)
    np.testing.assert_allclose(o.v[:, 0], [vcm, vcm], rtol=1e-13)


def test_oblique_collision_with_friction_closed_form():
    # single contact, no bias: lam_n = mt*(-u_n)_+, lam_t = -mt*u_t clipped to mu*lam_n
    m = mass(0.5)
    mt = m / 2.0
    for ut, mu in ((0.3, 0.5), (3.0, 0.5), (0.0, 0.2), (1.0, 0.0)):
        o = _two([0, 0, 0], [1, 0, 0], [1, ut, 0], [-1, 0, 0], n_iters=3, mu=mu)
        d = o.step(detail=True)
        ln = mt * 2.0                       # u_n = n.(v0 - v1) = -2 with n = -x
        lt = min(mt * ut, mu * ln)
        P = d["impulses"][0]
        np.testing.assert_allclose(P, [-ln, -lt, 0.0], rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(o.v[0], [1 - ln / m, ut - lt / m, 0], rtol=1e-13, atol=1e-15)


def test_sliding_sphere_on_plane_decelerates_by_mu_g_dt():
    g, dt, mu, u0 = 9.81, 1e-3, 0.5, 0.05
    r = float(np.float32(0.01))       # radius as binary32 so the gap is exactly 0
    o = O.Oracle(np.array([[0.0, 0.0, r]]), np.array([[u0, 0.0, 0.0]]), np.array([r], np.float32),
                 [scenes.plane((0, 0, 0), (0, 0, 1))], dt=dt, mu=mu, n_iters=20)
    for k in range(1, 16):
        o.step()
        expect = max(u0 - k * mu * g * dt, 0.0)
        assert abs(o.v[0, 0] - expect) < 1e-12
        assert abs(o.v[0, 2]) < 1e-12          # no vertical motion: resting contact
        assert abs(o.x[0, 2] - r) < 1e-12


@pytest.mark.parametrize("theta_deg", [10.0, 20.0, 26.0, 27.0, 35.0])
def test_incline_static_iff_tan_below_mu(theta_deg):
    g, dt, mu, r = 9.81, 1e-3, 0.5, float(np.float32(0.01))
    th = math.radians(theta_deg)
    nrm = np.array([-math.sin(th), 0.0, math.cos(th)])
    # a plane through the origin with unit normal nrm: rotate body z onto nrm
    t1 = np.array([math.cos(th), 0.0, math.sin(th)])
    R = np.stack([t1, np.cross(nrm, t1), nrm], axis=1)
    pl = scenes.plane((0, 0, 0), (0, 0, 1))
    pl["R"] = R
    # both sides see the pose in binary32: the effective incline is that of the
    # rounded rotation's third column
    n_eff = R.astype(np.float32).astype(np.float64)[:, 2]
    n_eff /= np.linalg.norm(n_eff)
    gv = np.array([0.0, 0.0, -g])
    g_n = -np.dot(gv, n_eff)
    g_t = np.linalg.norm(gv + g_n * n_eff)
    # a 1e-7 m overlap and no Baumgarte term: the contact persists through the
    # binary32 rounding of positions and the normal impulse only cancels gravity
    o = O.Oracle(np.array([nrm * (r - 1e-7)]), np.zeros((1, 3)), np.array([r], np.float32), [pl],
                 dt=dt, mu=mu, n_iters=20, alpha=0.0)
    speeds = []
    for k in range(10):
        o.step()
        speeds.append(float(np.linalg.norm(o.v[0])))
        assert abs(np.dot(o.v[0], n_eff)) < 1e-12
    if math.tan(th) <= mu:
        assert max(speeds) < 1e-9
    else:
        acc = g_t - mu * g_n
        np.testing.assert_allclose(speeds, [(k + 1) * acc * dt for k in range(10)], rtol=1e-9)


def test_free_fall_closed_form():
    dt = 1e-3
    x0 = np.array([[0.1, 0.2, 5.0], [1.0, 1.0, 7.0]])
    v0 = np.array([[0.3, -0.1, 2.0], [0.0, 0.5, 0.0]])
    o = O.Oracle(x0, v0, np.array([0.01, 0.01], np.float32), dt=dt)
    g = np.array([0, 0, -9.81])
    for k in range(1, 31):
        o.step()
        np.testing.assert_allclose(o.v, v0 + k * dt * g, rtol=0, atol=1e-12)
        np.testing.assert_allclose(o.x, x0 + k * dt * v0 + dt * dt * g * k * (k + 1) / 2, rtol=0, atol=1e-11)


def test_resting_column_stays_static():
    r = float(np.float32(0.005))
    n = 8
    x = np.array([[0.05, 0.05, r + 2 * r * k] for k in range(n)])
    o = O.Oracle(x, np.zeros((n, 3)), np.full(n, r, np.float32), [scenes.plane((0, 0, 0), (0, 0, 1))],
                 n_iters=20)
    x_start = o.x.copy()
    for _ in range(300):
        o.step()
    vmax = np.abs(o.v).max()
    assert vmax < 1e-3
    assert np.abs(o.x - x_start).max() < 1e-3 * r * 100   # settles within a tenth of r
    for _ in range(100):
        x_before = o.x.copy()
        o.step()
    assert np.abs(o.v).max() < 1e-4
    assert np.abs(o.x - x_before).max() < 1e-3 * r


def test_momentum_conserved_without_external_forces():
    rng = np.random.default_rng(7)
    x, r = scenes.random_spheres(300, ((0, 0.04), (0, 0.04), (0, 0.04)), 0.004, rng, r_jitter=0.3)
    v = rng.normal(size=(300, 3))
    o = O.Oracle(x.astype(np.float64), v, r, gravity=(0, 0, 0), n_iters=20, mu=0.4)
    m = np.array([mass(float(q)) for q in r])
    p0 = (m[:, None] * o.v).sum(0)
    d = o.step(detail=True)
    assert d["n_pp"] > 100
    p1 = (m[:, None] * o.v).sum(0)
    scale = (m[:, None] * np.abs(v)).sum()
    np.testing.assert_allclose(p1, p0, rtol=0, atol=1e-13 * scale)
    # impulses are equal and opposite: the accumulated dv carries no net momentum
    np.testing.assert_allclose((m[:, None] * d["dv"]).sum(0), 0, atol=1e-13 * scale)


def test_friction_cone_every_contact_every_iteration():
    s = scenes.drop_scene()
    o = O.scene_oracle(s, mu=0.3)
    for _ in range(40):
        o.step()
    d = o.step(detail=True, n_hist=20)
    H, nrm = d["history"], d["normals"]
    assert H.shape[1] > 500
    for l in range(H.shape[0]):
        ln = np.einsum("cd,cd->c", H[l], nrm)
        lt = np.linalg.norm(H[l] - ln[:, None] * nrm, axis=1)
        assert np.all(ln >= 0)
        assert np.all(lt <= 0.3 * ln * (1 + 1e-12) + 1e-300)


def test_order_independence():
    rng = np.random.default_rng(8)
    x, r = scenes.random_spheres(200, ((0, 0.03), (0, 0.03), (0, 0.03)), 0.004, rng)
    v = rng.normal(size=(200, 3)) * 0.1
    perm = rng.permutation(200)
    a = O.Oracle(x.astype(np.float64), v, r, [scenes.plane((0, 0, 0), (0, 0, 1))], n_iters=20)
    b = O.Oracle(x[perm].astype(np.float64), v[perm], r[perm], [scenes.plane((0, 0, 0), (0, 0, 1))], n_iters=20)
    a.step()
    b.step()
    np.testing.assert_allclose(b.v, a.v[perm], rtol=0, atol=1e-12)
    np.testing.assert_allclose(b.x, a.x[perm], rtol=0, atol=1e-14)


def _lcp_by_enumeration(A, q):
    """Frictionless NCP of Eqs. (1)-(2): 0 <= lam  _|_  A lam + q >= 0,
    solved by trying every active set (textbook enumeration, tiny systems)."""
    m = len(q)
    best = None
    for k in range(m + 1):
        for S in itertools.combinations(range(m), k):
            lam = np.zeros(m)
            if S:
                S = list(S)
                sol, *_ = np.linalg.lstsq(A[np.ix_(S, S)], -q[S], rcond=None)
                lam[S] = sol
            c = A @ lam + q
            if lam.min() >= -1e-9 and c.min() >= -1e-9:
                best = lam
                return best
    return best


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_frictionless_limit_is_lcp_solution(seed):
    rng = np.random.default_rng(seed)
    # a small cluster of overlapping spheres (a random chain with overlapping
    # links) with random velocities, no gravity
    n = 5
    r = 0.5
    x = np.zeros((n, 3))
    for k in range(1, n):
        d = rng.normal(size=3)
        x[k] = x[k - 1] + 0.97 * d / np.linalg.norm(d)
    x = x.astype(np.float32).astype(np.float64)
    v = rng.normal(size=(n, 3))
    rr = np.full(n, r, np.float32)
    pairs = O.pp_bruteforce(x.astype(np.float32), rr)
    if not (1 <= len(pairs) <= 8):
        pytest.skip("cluster outside 1..8 contacts for this seed")
    dt, alpha = 1e-2, 0.2
    m = mass(r)
    # J rows: contact normal (from j to i) acting on i (+) and j (-), computed here
    Cn = len(pairs)
    J = np.zeros((Cn, 3 * n))
    bias = np.zeros(Cn)
    for c, (i, j) in enumerate(pairs):
        d = x[i] - x[j]
        L = np.linalg.norm(d)
        nc = d / L
        J[c, 3 * i:3 * i + 3] = nc
        J[c, 3 * j:3 * j + 3] = -nc
        bias[c] = alpha * (L - 2 * r) / dt
    Minv = np.eye(3 * n) / m
    A = J @ Minv @ J.T
    q = J @ v.reshape(-1) + bias
    lam = _lcp_by_enumeration(A, q)
    assert lam is not None
    w_ref = v.reshape(-1) + Minv @ J.T @ lam
    o = O.Oracle(x, v, rr, gravity=(0, 0, 0), dt=dt, alpha=alpha, mu=0.0, n_iters=20000)
    o.step()
    np.testing.assert_allclose(o.v.reshape(-1), w_ref, rtol=0, atol=1e-7 * (1 + np.abs(v).max()))


@pytest.mark.parametrize("split", [True, False])
def test_mass_splitting_iterates_closed_form(split):
    # particle 0 at rest hit head-on from both sides at speed u.  With mass
    # splitting (n_0 = 2, n_1 = n_2 = 1) mt = m/3 and the iterates obey
    # w_1(l) = (2/3) w_1(l-1); without it mt = m/2 and w_1(l) = (1/2) w_1(l-1).
    # w_0 stays 0 by symmetry.
    u = 1.0
    x = np.array([[-1.0, 0, 0], [0.0, 0, 0], [1.0, 0, 0]])
    # order: particle 0 is the middle one in the test's naming -> index 1 here
    v = np.array([[u, 0, 0], [0, 0, 0], [-u, 0, 0]])
    ratio = 2.0 / 3.0 if split else 0.5
    for iters in (1, 2, 3, 7):
        o = O.Oracle(x, v, np.full(3, 0.5, np.float32), gravity=(0, 0, 0), n_iters=iters,
                     mass_split=split, mu=0.5)
        o.step()
        np.testing.assert_allclose(o.v[0], [u * ratio ** iters, 0, 0], rtol=1e-13)
        np.testing.assert_allclose(o.v[2], [-u * ratio ** iters, 0, 0], rtol=1e-13)
        np.testing.assert_allclose(o.v[1], 0, atol=1e-15)


def test_body_advance_matches_scipy_rotation():
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(9)
    R0 = scenes.random_rotation(rng)
    om = np.array([0.3, -1.2, 0.7])
    nu = np.array([0.1, 0.0, -0.2])
    cap = scenes.capsule_tool((0.1, 0.2, 0.3), 0.02, 0.075, nu=nu, omega=om, R=R0)
    B = O.make_bodies([cap])
    dt = 1e-3
    for _ in range(100):
        O.lib().ggo_advance_bodies(1, B, dt)
    R = np.array(B[0].R[:]).reshape(3, 3)
    Rref = Rotation.from_rotvec(om * dt * 100).as_matrix() @ R0
    np.testing.assert_allclose(R, Rref, atol=1e-12)
    np.testing.assert_allclose(np.array(B[0].t[:]), np.array([0.1, 0.2, 0.3]) + 100 * dt * nu, atol=1e-14)


def test_body_point_velocity_of_rotating_tool():
    # a sphere resting on a plane that translates up at 0.1 m/s: after one step
    # the contact drives the normal relative velocity to zero, so v_z = 0.1.
    r = float(np.float32(0.01))
    pl = scenes.plane((0, 0, 0), (0, 0, 1))
    pl["nu"] = np.array([0.0, 0.0, 0.1])
    o = O.Oracle(np.array([[0.0, 0.0, r]]), np.zeros((1, 3)), np.array([r], np.float32), [pl],
                 n_iters=5, alpha=0.0)
    o.step()
    assert abs(o.v[0, 2] - float(np.float32(0.1))) < 1e-12   # body twist is handed over in binary32


def test_cyclic_vertical_boundary_closed_form():
    # no gravity, no contacts, downward velocities: with the tower's cyclic
    # boundary the height is periodic, z_k = lo + ((z_0 + k dt v - lo) mod H)
    # (floored modulus), velocities unchanged
    n, dt, steps = 20, 1e-3, 400
    rng = np.random.default_rng(4)
    x = np.column_stack([np.arange(n) * 0.01, np.zeros(n), rng.uniform(0.05, 0.45, n)])
    v = np.zeros((n, 3))
    v[:, 2] = -rng.uniform(1.0, 3.0, n)
    lo, hi = 0.0, 0.5
    orc = O.Oracle(x, v, np.full(n, 0.001, np.float32), [], dt=dt, gravity=(0.0, 0.0, 0.0), cyclic_z=(lo, hi))
    for _ in range(steps):
        orc.step()
    z = lo + np.mod(x[:, 2] + steps * dt * v[:, 2] - lo, hi - lo)
    np.testing.assert_allclose(orc.x[:, 2], z, rtol=0, atol=1e-11)
    np.testing.assert_array_equal(orc.v, v)
    assert np.all(steps * dt * v[:, 2] < -(hi - lo) * 0.8)    # every grain wrapped at least once


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def test_turntable_carries_a_sticking_sphere_at_the_rigid_velocity():
    # A plane spinning about the vertical axis through (a, b, 0) (an se(3)
    # twist with nu = 0, omega = Omega z, Sec. II) under a sphere resting on it
    # at (rho, 0, r).  The contact point is (rho, 0, 0), so the body point
    # velocity is omega x (p_c - t) = Omega (b, rho - a, 0).  With gravity
    # pressing the sphere down, one step makes it move with that point as long
    # as Omega |arm| <= mu g dt (sticking); beyond, the tangential impulse is
    # capped at mu m g dt and the sphere slides along the point velocity at
    # speed mu g dt (disk projection of Alg. 1).
    g, dt, mu = 9.81, 1e-3, 0.5
    r = float(np.float32(0.01))
    a, b, rho = 0.25, -0.125, 0.5
    arm = math.hypot(rho - a, b)
    for Omega, sticking in ((0.5 * mu * g * dt / arm, True), (0.9 * mu * g * dt / arm, True),
                            (4.0 * mu * g * dt / arm, False), (-3.0 * mu * g * dt / arm, False)):
        Om = float(np.float32(Omega))
        pl = scenes.plane((a, b, 0.0), (0, 0, 1))
        pl["omega"] = np.array([0.0, 0.0, Om])
        o = O.Oracle(np.array([[rho, 0.0, r]]), np.zeros((1, 3)), np.array([r], np.float32), [pl],
                     dt=dt, mu=mu, n_iters=20, alpha=0.0)
        d = o.step(detail=True)
        assert d["n_pb"] == 1
        V = Om * np.array([b, rho - a, 0.0])
        if sticking:
            np.testing.assert_allclose(o.v[0], V, rtol=0, atol=1e-15)
        else:
            expect = mu * g * dt * V / np.linalg.norm(V)
            np.testing.assert_allclose(o.v[0], expect, rtol=0, atol=1e-15)
        # the normal impulse carries the weight exactly: no vertical motion
        assert abs(o.v[0, 2]) < 1e-15


def test_pushing_body_imparts_its_rigid_point_velocity():
    # A body pushing a free sphere (no gravity, no Baumgarte bias) within the
    # friction cone: after one sweep the sphere moves with the body's rigid
    # velocity at the contact point, V = nu + omega x (p_c - t), where
    # p_c = x - f n is the point of the surface under the sphere centre (the
    # body contact geometry of Eq. (7)), and later sweeps keep that fixed
    # point.  The rotation is generic, so omega is not parallel to the normal
    # and using the sphere centre x instead of p_c, or the opposite sign of the
    # cross product, would change V.
    rng = np.random.default_rng(21)
    r = float(np.float32(0.01))
    mu = 0.5
    checked = 0
    for trial in range(12):
        R = scenes.random_rotation(rng)
        t = rng.uniform(-0.2, 0.2, 3)
        Rf, tf = _f32(R), _f32(t)
        n = Rf[:, 2] / np.linalg.norm(Rf[:, 2])
        om = _f32(rng.uniform(-1.0, 1.0, 3))
        nu = _f32(1.0 * n + rng.uniform(-0.05, 0.05, 3))
        pb = np.array([rng.uniform(-0.1, 0.1), rng.uniform(-0.1, 0.1), r * (1 - 1e-3)])
        x = tf + Rf @ pb
        body = {"shape": "plane", "params": [0.0] * 4, "R": R, "t": t, "nu": nu, "omega": om, "env": 0}
        for iters in (1, 3):
            o = O.Oracle(x[None, :], np.zeros((1, 3)), np.array([r], np.float32), [body],
                         gravity=(0.0, 0.0, 0.0), alpha=0.0, mu=mu, n_iters=iters)
            d = o.step(detail=True)
            assert d["n_pb"] == 1
            f = float(np.dot(Rf.T @ (x - tf), [0, 0, 1.0]))
            pc = x - f * n
            V = nu + np.cross(om, pc - tf)
            Vn = float(V @ n)
            Vt = V - Vn * n
            assert Vn > 0 and np.linalg.norm(Vt) <= mu * Vn      # the sticking regime
            np.testing.assert_allclose(o.v[0], V, rtol=0, atol=1e-12)
            # x instead of p_c shifts the arm by f n: a different velocity
            assert np.linalg.norm(np.cross(om, f * n)) > 1e-4
            checked += 1
    assert checked == 24


@pytest.mark.parametrize("relax", [0.3, 0.7, 1.3])
def test_relaxed_sweeps_decay_the_relative_velocity_geometrically(relax):
    # Two equal spheres touching head on (no gravity), approaching with a
    # relative velocity u0 inside the friction cone.  Every sweep's projected
    # value is the full inelastic impulse y = -mt u0 (mt = m/2), so the blend
    # lam_l = (1 - w) lam_{l-1} + w y leaves lam* - lam_l = (1 - w)^l lam*, and
    # the relative velocity after I sweeps is (1 - w)^I u0, both along the
    # normal and (sticking) along the tangent.  Momentum is unchanged.
    m = mass(0.5)
    v0 = np.array([[1.0, 0.2, -0.1], [-1.0, 0.0, 0.1]])
    for iters in (1, 2, 5, 9):
        o = _two([0, 0, 0], [1, 0, 0], v0[0], v0[1], n_iters=iters, mu=0.5, relax=relax)
        o.step()
        u0 = v0[0] - v0[1]
        np.testing.assert_allclose(o.v[0] - o.v[1], (1.0 - relax) ** iters * u0, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(m * (o.v[0] + o.v[1]), m * (v0[0] + v0[1]), rtol=1e-13, atol=1e-13)
