"""Pins for the oracle's post-processing: pressure at points of the fluid from the
surface pressure (eq. (cbie) with c = 1) and the insertion loss (eq. (insertionloss))."""
import numpy as np
import pytest

from oracle import bem, mie, solve
from workloads import Lattice, icosphere

ONE_CELL = Lattice((1, 1, 1), (0.3, 0.3, 0.3))


def test_gauss_solid_angle_at_k0():
    # at k = 0 the double-layer potential of p = 1 over a closed surface is the solid angle
    # it subtends over 4 pi: 1 inside (normals point into the scatterer), 0 outside
    v, t = icosphere(2, 0.1)
    inside = np.array([[0.0, 0.0, 0.0], [0.03, 0.02, -0.01], [-0.05, 0.04, 0.02]])
    outside = np.array([[0.3, 0.0, 0.0], [0.12, 0.05, 0.0], [0.0, 0.0, -0.5]])
    W = bem.field_weights(v, t, ONE_CELL, 0.0, np.vstack([inside, outside]))
    s = W.sum(1)
    assert np.allclose(s[:3], 1.0, atol=1e-9)
    assert np.allclose(s[3:], 0.0, atol=1e-9)


def test_gauss_solid_angle_over_lattice_cells():
    # the same invariant with the surface spread over a lattice: each cell's sphere counts
    # once, so a point inside the sphere of cell c gets 1 from that cell and 0 from others
    v, t = icosphere(1, 0.1)
    lat = Lattice((3, 2, 1), (0.3, 0.25, 0.3))
    pts = np.array([lat.cell_origin(4) + [0.01, -0.02, 0.0], [0.15, 0.125, 0.0], [0.6, 0.25, 0.2]])
    W = bem.field_weights(v, t, lat, 0.0, pts)
    n = t.shape[0]
    per_cell = W.reshape(3, lat.n_cells, n).sum(-1)
    expect = np.zeros((3, lat.n_cells))
    expect[0, 4] = 1.0
    assert np.allclose(per_cell, expect, atol=1e-9)


def _sphere_fields(level, formulation, f=500.0):
    v, t = icosphere(level, 0.1)
    k = 2 * np.pi * f / 343.0
    a = bem.default_alpha(k, formulation)
    x = solve.lu_solve(bem.dense_exact(v, t, ONE_CELL, k, a),
                       bem.rhs_plane_wave(v, t, ONE_CELL, k, a, [[1.0, 0.0, 0.0]])[0])
    rng = np.random.default_rng(3)
    d = rng.normal(size=(12, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    out_pts = d * np.array([0.15, 0.2, 0.3, 0.5] * 3)[:, None]
    in_pts = np.array([[0.0, 0.0, 0.0], [0.02, 0.03, 0.01], [-0.04, 0.0, 0.02]])
    pts = np.vstack([out_pts, in_pts])
    pin = bem.incident_plane_wave_at(pts, k, [[1.0, 0.0, 0.0]])[0]
    p = bem.field(v, t, ONE_CELL, k, pts, x, pin)
    ex = mie.rigid_sphere_total_field(out_pts, 0.1, k)
    scat_err = np.linalg.norm((p[:12] - pin[:12]) - (ex - pin[:12])) / np.linalg.norm(ex - pin[:12])
    return scat_err, np.abs(p[12:]).max()


@pytest.mark.parametrize("formulation", ["bm", "cbie"])
def test_field_converges_to_mie(formulation):
    # outside the sphere the field converges to the exterior Mie series (O(h^2), ~3.7x per
    # level); inside, the representation gives zero (extinction), which fixes the sign of
    # the double-layer term: the wrong sign leaves 2 p_inc there.  Bounds calibrated once.
    e1, z1 = _sphere_fields(1, formulation)
    e2, z2 = _sphere_fields(2, formulation)
    assert e2 < e1 / 3.0
    assert e1 < 0.1 and e2 < 0.03
    assert z2 < z1 and z2 < 0.005


def test_mie_total_field_reduces_to_surface_pressure():
    # at r = a the exterior series equals the Wronskian form of the surface pressure
    rng = np.random.default_rng(5)
    d = rng.normal(size=(6, 3))
    pts = 0.1 * d / np.linalg.norm(d, axis=1)[:, None]
    k = 2 * np.pi * 700.0 / 343.0
    assert np.allclose(mie.rigid_sphere_total_field(pts, 0.1, k), mie.rigid_sphere_surface_pressure(pts, 0.1, k),
                       atol=1e-12)


@pytest.mark.parametrize("which", ["plane", "point"])
def test_incident_fields_solve_helmholtz(which):
    # second-order central differences: |lap p + k^2 p| = O(h^2 k^4 |p|)
    k = 2 * np.pi * 800.0 / 343.0
    x0 = np.array([[0.31, -0.12, 0.4], [1.2, 0.5, -0.3]])
    h = 1e-3
    def p(x):
        if which == "plane":
            return bem.incident_plane_wave_at(x, k, [[0.6, 0.0, 0.8]], 2.0)[0]
        return bem.incident_point_source_at(x, k, [[0.0, -2.0, 0.9]], 2.0)[0]
    lap = -6.0 * p(x0)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        lap += p(x0 + e) + p(x0 - e)
    lap /= h * h
    assert np.all(np.abs(lap + k * k * p(x0)) < 1e-4 * k * k * np.abs(p(x0)))


def test_point_source_amplitude_and_phase():
    # |p| = A / R and phase k R at distance R (outgoing wave, e^{-i w t})
    k = 3.0
    p = bem.incident_point_source_at([[0.0, 0.0, 2.0]], k, [[0.0, 0.0, 0.0]], 1.5)[0, 0]
    assert np.isclose(abs(p), 0.75) and np.isclose(np.angle(p), k * 2.0 - 2 * np.pi)


def test_insertion_loss_closed_forms():
    rng = np.random.default_rng(1)
    pin = rng.normal(size=(2, 64)) + 1j * rng.normal(size=(2, 64))
    assert np.allclose(bem.insertion_loss(pin, pin), 0.0)
    assert np.allclose(bem.insertion_loss(pin, 0.1 * pin * np.exp(1j * rng.uniform(size=64))), 20.0)
    assert np.isclose(bem.insertion_loss(pin[0], 0.5 * pin[0]), 20 * np.log10(2.0))
