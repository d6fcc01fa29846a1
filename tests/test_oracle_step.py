"""Pins of the oracle's projection step (no GPU).

P-PRJ1 : EXTENDED mode - the projected spectrum is divergence-free on the
         extended periodic lattice: sum_a S_a u_hat_a = 0 to round-off.
P-PRJ2 : all-periodic lattice, PHYSICAL mode with SPH eigenvalues - the new
         velocity has zero SPH divergence to round-off (the PPE inverts exactly
         the operator div o grad of the method), and a velocity that is already
         discretely divergence-free is left unchanged.
Walls  : Dirichlet wall points of the new velocity carry the wall data.
Modes  : the direct (tap sum) and FFT operator modes give the same step.
"""
import numpy as np

from oracle import operators, step
from oracle.lattice import Lattice, walled_box
from paper_2606_06247_amd import synth


def test_extended_projection_divergence_free(fc_tables):
    lat = walled_box((24, 24))
    u = [synth.poly_trig_2d(24, seed=s) for s in (0, 1)]
    unew, phi, parts = step.project_step(lat, fc_tables, u, dt=1e-3, nu=1e-3, mode="extended",
                                         return_parts=True)
    S = parts["S"]
    div_new = sum(S[a] * parts["uhat_new"][a] for a in range(2))
    assert np.max(np.abs(div_new)) < 1e-13 * np.max(np.abs(parts["D"]))


def test_periodic_sph_projection_divergence_free():
    lat = Lattice(n=(20, 16), walled=(False, False), dx=1.0 / 20)
    ops = operators.Operators(lat, None)
    rng = np.random.default_rng(11)
    u = [rng.standard_normal((16, 20)) for _ in range(2)]
    unew, phi = step.project_step(lat, None, u, dt=1e-3, nu=1e-2, family="sph")
    dnew = ops.div(unew)
    dstar = ops.div(step.project_step(lat, None, u, dt=1e-3, nu=1e-2, family="sph",
                                      return_parts=True)[2]["ustar"])
    assert np.max(np.abs(dnew)) < 1e-11 * np.max(np.abs(dstar))
    # an already divergence-free field (grad-perp of a stream function) is kept
    psi = rng.standard_normal((16, 20))
    gp = ops.grad(psi)
    v = [gp[1], -gp[0]]        # (d psi/dy, -d psi/dx): SPH-divergence-free
    assert np.max(np.abs(ops.div(v))) < 1e-10 * np.max(np.abs(v[0]))


def test_dirichlet_walls_and_mode_agreement(fc_tables):
    n = 21
    lat = walled_box((n, n), vel_bc=(("D", "N"), ("D", "D")))
    u = [synth.poly_trig_2d(n, seed=s) for s in (3, 4)]
    f = [synth.poly_trig_2d(n, seed=s) for s in (5, 6)]
    w = [synth.poly_trig_2d(n, seed=s) for s in (7, 8)]
    a, pa = step.project_step(lat, fc_tables, u, force=f, wall=w, dt=1e-4, nu=1e-3)
    b, pb = step.project_step(lat, fc_tables, u, force=f, wall=w, dt=1e-4, nu=1e-3, opmode="fft")
    for c in range(2):
        assert np.array_equal(a[c][:, 0], w[c][:, 0])      # x low wall (D)
        assert not np.array_equal(a[c][:, -1], w[c][:, -1])  # x high wall (N)
        assert np.array_equal(a[c][0, :], w[c][0, :])      # y walls (D)
        assert np.array_equal(a[c][-1, :], w[c][-1, :])
        assert np.max(np.abs(a[c] - b[c])) < 1e-10 * np.max(np.abs(a[c]))
    assert np.max(np.abs(pa - pb)) < 1e-10 * np.max(np.abs(pa))


def test_zero_state_stays_zero(fc_tables):
    lat = walled_box((16, 16))
    z = [np.zeros((16, 16)), np.zeros((16, 16))]
    un, p = step.project_step(lat, fc_tables, z)
    assert all(np.max(np.abs(c)) == 0 for c in un) and np.max(np.abs(p)) == 0


def test_channel_3d_projection_walls_and_modes(fc_tables):
    """The 3D channel lattice: P-PRJ1 in EXTENDED mode, Dirichlet walls and
    the direct / FFT operator modes in PHYSICAL mode."""
    n = (12, 17, 10)
    lat = Lattice(n=n, walled=(False, True, False), dx=1.0 / 16, vel_bc=(None, ("D", "D"), None),
                  prs_bc=(None, ("N", "N"), None))
    u = synth.ChannelFlow3D(n, 1, 2).u
    f = synth.ChannelFlow3D(n, 3, 4).u
    w = [c + 0.25 for c in synth.ChannelFlow3D(n, 5, 6).u]
    unew, phi, parts = step.project_step(lat, fc_tables, u, force=f, wall=w, dt=1e-3, nu=1e-3,
                                         mode="extended", return_parts=True)
    S = parts["S"]
    div_new = sum(S[a] * parts["uhat_new"][a] for a in range(3))
    assert np.max(np.abs(div_new)) < 1e-13 * np.max(np.abs(parts["D"]))
    a, pa = step.project_step(lat, fc_tables, u, force=f, wall=w, dt=1e-4, nu=1e-3)
    b, pb = step.project_step(lat, fc_tables, u, force=f, wall=w, dt=1e-4, nu=1e-3, opmode="fft")
    for c in range(3):
        assert np.array_equal(a[c][:, 0, :], w[c][:, 0, :])
        assert np.array_equal(a[c][:, -1, :], w[c][:, -1, :])
        assert np.max(np.abs(a[c] - b[c])) < 1e-10 * np.max(np.abs(a[c]))
    assert np.max(np.abs(pa - pb)) < 1e-10 * np.max(np.abs(pa))
