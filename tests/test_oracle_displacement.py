"""Pins of the oracle's displacement form (CPU only).

With ``displacement=True`` the marker state is D = X - X_ref: positions are
formed as X_ref + D only where the delta function is evaluated, and the
elastic terms are written in D, so that strains far below the rounding of
O(1) positions keep their own relative precision.  The mathematics is the
same as in the position form, so the two must agree wherever the position
form is itself accurate, and the displacement form must have the exact
structure the energies give it (bending and tethers are linear in D).
"""
import numpy as np
import pytest

from paper_math_0301321_amd import workloads as W


def _models(oracle_mod, wl):
    return oracle_mod.Model(wl), oracle_mod.Model(wl, displacement=True)


def test_force_agrees_with_the_position_form(oracle_mod):
    """Strains of 1e-2 (where positions resolve them to ~1e-12): the two forms'
    forces agree to 1e-9 of the largest, with springs, lattices, tethers and
    the drive all present."""
    for wl in (W.tiny_helix(window=12), W.config1()):
        mx, md = _models(oracle_mod, wl)
        rng = np.random.default_rng(5)
        D = 1e-2 * wl.h * rng.standard_normal(wl.X0.shape) + (wl.X0 - wl.X_ref)
        X = wl.X_ref + D
        for t in (0.0, 3.7e-4):
            Fx = oracle_mod.force(mx, X, t)
            Fd = oracle_mod.force(md, D, t)
            assert np.abs(Fd - Fx).max() <= 1e-9 * np.abs(Fx).max(), (wl.name, t)


def test_force_vanishes_at_zero_displacement(oracle_mod):
    wl = W.tiny_helix(window=12)
    md = oracle_mod.Model(wl, displacement=True)
    assert np.count_nonzero(oracle_mod.force(md, np.zeros_like(wl.X0), 0.0)) == 0


def test_bend_and_tether_forces_are_linear_in_the_displacement(oracle_mod):
    """The bend energy is quadratic in the second difference of D and the tether
    energy in D itself, so their forces are exactly linear in D: at nm
    displacements (1e-9 of the O(1) positions) F(3D) = 3 F(D) to rounding of
    the forces themselves.  The position form resolves the same second
    differences only to ~1e-16 / 1e-13 of their size."""
    wl = W.tiny_helix()
    for lat in wl.lattices:
        lat.Ks = 0.0                                  # bending and tethers only
    md = oracle_mod.Model(wl, displacement=True)
    rng = np.random.default_rng(6)
    D = 1e-9 * rng.standard_normal(wl.X0.shape)
    F1 = oracle_mod.force(md, D, 0.0)
    F3 = oracle_mod.force(md, 3.0 * D, 0.0)
    assert np.abs(F1).max() > 0
    assert np.abs(F3 - 3.0 * F1).max() <= 1e-13 * np.abs(F3).max()


def test_stretch_at_tiny_strain_matches_the_closed_form(oracle_mod):
    """One lattice edge stretched by a strain of 1e-12 (far below the relative
    rounding of the positions): in the displacement form the force is the
    closed form Ks kbar wbar eps / Le along the edge to 1e-10, since the
    extension is formed from the displacement difference."""
    Ks, Le, eps = 50.0, 0.01, 1e-12
    k, w = np.array([1.0, 3.0]), np.array([0.2, 0.6])
    e = np.array([2.0, -1.0, 2.0]) / 3.0
    ya = np.array([0.31, 0.52, 0.47])
    Y = np.stack([ya, ya + Le * e], axis=1)
    D = np.zeros((3, 2))
    D[:, 1] = eps * Le * e
    wl = W.Workload(name="edge", N=16, L=1.0, rho=1.0, mu=0.01, dt=1e-4, n_steps=1, convect=0,
                    X0=Y + D, w=w, k=k, X_ref=Y, kappa=np.zeros(2), lattices=[W.Lattice(0, 2, 1, False, Ks, 0.0)],
                    spring_ab=np.zeros((2, 0), np.int32), spring_rest=np.zeros(0), K_spring=0.0,
                    drive_idx=np.zeros(0, np.int32), drive_dir=np.zeros((3, 0)), drive_A=0.0, drive_freq=0.0)
    F = oracle_mod.force(oracle_mod.Model(wl, displacement=True), D, 0.0)
    mag = Ks * 2.0 * 0.4 * eps / Le
    np.testing.assert_allclose(F[:, 1], -mag * e, rtol=1e-10, atol=0)
    np.testing.assert_allclose(F[:, 0], mag * e, rtol=1e-10, atol=0)


def test_positions_are_reference_plus_displacement(oracle_mod):
    wl = W.tiny_helix()
    md = oracle_mod.Model(wl, displacement=True)
    rng = np.random.default_rng(7)
    D = 1e-4 * rng.standard_normal(wl.X0.shape)
    assert np.array_equal(oracle_mod.positions(md, D), wl.X_ref + D)
    mx = oracle_mod.Model(wl)
    assert np.array_equal(oracle_mod.positions(mx, wl.X0), wl.X0)


@pytest.mark.parametrize("convect", [0, 1])
def test_trajectory_agrees_with_the_position_form(oracle_mod, convect):
    """Ten steps of the tiny helix from rest: the displacement form's D^n and the
    position form's X^n - X_ref agree to 1e-9 of the largest displacement (the
    position form's own rounding of displacements on O(1) positions), and so do
    the velocities."""
    wl = W.tiny_helix()
    wl.convect = convect
    Xx, ux = oracle_mod.run(wl, 10)
    Dd, ud = oracle_mod.run(wl, 10, displacement=True)
    dX = Xx - wl.X_ref
    assert np.abs(dX).max() > 0
    assert np.abs(Dd - dX).max() <= 1e-9 * np.abs(dX).max()
    assert np.abs(ud - ux).max() <= 1e-9 * np.abs(ux).max()


@pytest.mark.parametrize("convect", [0, 1])
def test_adjoint_step_is_transpose_of_linearised_step(oracle_mod, convect):
    """The displacement form's adjoint step against central differences of its
    own forward step, as for the position form."""
    wl = W.tiny_helix(N=16)
    wl.convect = convect
    rng = np.random.default_rng(31)
    D = 2e-3 * rng.standard_normal(wl.X0.shape)
    u = 0.05 * W.random_field(16, seed=32)
    t = 3e-4
    dD, du, dk = rng.standard_normal(D.shape), rng.standard_normal(u.shape), rng.standard_normal(wl.M)
    Db1, ub1 = rng.standard_normal(D.shape), rng.standard_normal(u.shape)

    def fwd(e):
        m = oracle_mod.Model(wl, wl.k + e * dk, displacement=True)
        return oracle_mod.step(m, wl, D + e * dD, u + e * du, t, convect=convect)

    eps = 1e-6
    Dp, up = fwd(eps)
    Dm, um = fwd(-eps)
    lhs = ((Dp - Dm) / (2 * eps) * Db1).sum() + ((up - um) / (2 * eps) * ub1).sum()
    m = oracle_mod.Model(wl, displacement=True)
    _, u1 = oracle_mod.step(m, wl, D, u, t, convect=convect)
    Db, ub, kb = oracle_mod.adjoint_step(m, wl, D, u1, t, Db1, ub1, np.zeros(wl.M), convect=convect, u_n=u)
    rhs = (dD * Db).sum() + (du * ub).sum() + (dk * kb).sum()
    assert abs(lhs - rhs) <= 1e-6 * abs(rhs), (lhs, rhs)


def test_nm_gradient_against_finite_differences(oracle_mod):
    """Where the position form cannot resolve the strains (micrometre motion on
    O(1) positions: its central differences of single stiffnesses scatter by
    1e-2 .. 1 about the adjoint for eps from 1e-7 to 1e-3), the displacement
    form's reverse-mode stiffness gradient agrees with central differences of
    single stiffnesses at a relative eps = 1e-2 to 1e-4 of the larger of
    |g_fd| and 1e-3 max |g_fd| (measured 3e-8 .. 4e-5).  Smaller eps are
    limited by the loss's own FP64 rounding (about 1e-14 of it here): a
    marker whose influence k_i dL/dk_i is 1e-8 of L needs eps ~ 1e-2 to rise
    above it."""
    wl = W.tiny_helix(N=16)
    wl.convect = 0
    idx = W.bm_index(wl, np.arange(20, 40), np.arange(wl.meta["bm_across"]))
    n = 8
    L0, g, _, _ = oracle_mod.gradient_k(wl, n, idx, displacement=True)
    assert L0 > 0

    def loss(k):
        D, _ = oracle_mod.run(wl, n, k=k, convect=0, displacement=True)
        d = D[:, idx]
        return (d * d).sum() / len(idx)

    assert abs(loss(wl.k) - L0) <= 1e-12 * L0
    rng = np.random.default_rng(1)
    nb = W.bm_count(wl)
    gmax = np.abs(g[:nb]).max()
    for i in rng.choice(nb, 6, replace=False):
        e = 1e-2 * wl.k[i]
        kp, km = wl.k.copy(), wl.k.copy()
        kp[i] += e
        km[i] -= e
        gfd = (loss(kp) - loss(km)) / (2 * e)
        assert abs(g[i] - gfd) <= 1e-4 * max(abs(gfd), 1e-3 * gmax), (i, g[i], gfd)
