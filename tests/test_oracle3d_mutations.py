"""Plant plausible mistakes in the 3-D oracle (on the CPU, in the oracle only)
and check that a pin catches each."""
import numpy as np
import pytest

import pins3d
from oracle import felbm3d_oracle as fo3

_lapC, _lapmu, _wall, _rhs, _pf, _eq = fo3.laplacian_C, fo3.laplacian_mu, fo3.wall_flux, fo3.rhs, fo3.point_forces, \
    fo3.equilibria
_Geometry = fo3.Geometry


class GeometryTwoThirds(_Geometry):
    """|f| n = -2 V grad N (the triangle's factor) instead of -3 V grad N."""

    def __init__(self, mesh):
        super().__init__(mesh)
        self.face_area_vec = self.face_area_vec * (2.0 / 3.0)


def lapmu_doubled(geo, gradmu):
    return 2.0 * _lapmu(geo, gradmu)


def lapC_no_average(geo, C, gradC, bc):
    saved = geo.face_nbr.copy()
    geo.face_nbr[:] = np.where(saved >= 0, np.arange(geo.NT)[:, None], saved)
    try:
        return _lapC(geo, C, gradC, bc)
    finally:
        geo.face_nbr[:] = saved


def wall_flux_trapezoid(Cf, rf, area):
    # the cubic integrand by the vertex rule instead of exactly
    return -area / 3.0 * sum(rf[i] * (Cf[i] - Cf[i] * Cf[i]) for i in range(3))


def lapC_no_incident_wall_faces(geo, C, gradC, bc):
    saved, sa = geo.wall_faces, geo.wall_area
    geo.wall_faces, geo.wall_area = saved[:0], sa[:0]
    try:
        return _lapC(geo, C, gradC, bc)
    finally:
        geo.wall_faces, geo.wall_area = saved, sa


def rhs_printed_sign(mat, dt, psi_hat, Phi):
    out = _rhs(mat, dt, psi_hat, np.zeros_like(Phi))
    return out + np.stack([-dt * (mat.M10 @ Phi[:, a]) + dt * dt * (mat.Ka[a] @ Phi[:, a]) for a in range(fo3.Q)], 1)


def rhs_no_D(mat, dt, psi_hat, Phi):
    return np.stack([-dt * (mat.Ca[a] @ psi_hat[:, a]) + dt * (mat.M10 @ Phi[:, a]) + dt * dt * (mat.Ka[a] @ Phi[:, a])
                     for a in range(fo3.Q)], 1)


def rhs_K_sign(mat, dt, psi_hat, Phi):
    return np.stack([-dt * (mat.Ca[a] @ psi_hat[:, a]) - dt * dt * (mat.Da[a] @ psi_hat[:, a])
                     + dt * (mat.M10 @ Phi[:, a]) - dt * dt * (mat.Ka[a] @ Phi[:, a]) for a in range(fo3.Q)], 1)


def rhs_C_transposed(mat, dt, psi_hat, Phi):
    return np.stack([-dt * (mat.Ca[a].T @ psi_hat[:, a]) - dt * dt * (mat.Da[a] @ psi_hat[:, a])
                     + dt * (mat.M10 @ Phi[:, a]) + dt * dt * (mat.Ka[a] @ Phi[:, a]) for a in range(fo3.Q)], 1)


def wall_flux_flipped(Cf, rf, area):
    return -_wall(Cf, rf, area)


def forces_no_mobility(prm, C, rho, u, mu, gradC, gradp, gradrho, lapmu):
    return _pf(prm, C, rho, u, mu, gradC, gradp, gradrho, 0 * lapmu)


def _h_force(eq_h_term):
    """point_forces with the X vector of eq:H replaced by eq_h_term(C, rho, mu, gradC, gradp)."""
    def forces(prm, C, rho, u, mu, gradC, gradp, gradrho, lapmu):
        Pg, _ = _pf(prm, C, rho, u, mu, gradC, gradp, gradrho, lapmu)
        Gu = fo3.gamma(u)
        X = eq_h_term(C, rho, mu, gradC, gradp)
        return Pg, (fo3.edot(X) - np.sum(u * X, axis=1)[:, None]) * Gu + prm.mobility * lapmu[:, None] * Gu
    return forces


eqH_term_deleted = _h_force(lambda C, rho, mu, gC, gp: gC)
eqH_mu_sign = _h_force(lambda C, rho, mu, gC, gp: gC - (C / (rho * fo3.CS2))[:, None] * (gp + mu[:, None] * gC))
eqH_rho_one = _h_force(lambda C, rho, mu, gC, gp: gC - (C / fo3.CS2)[:, None] * (gp - mu[:, None] * gC))


def gamma_quadratic_doubled(u):
    eu = fo3.edot(u)
    uu = np.sum(u * u, axis=1)[:, None]
    return fo3.W * (1.0 + eu / fo3.CS2 + (eu * eu - fo3.CS2 * uu) / (fo3.CS2 * fo3.CS2))


def g_eq_quadratic_doubled(C, p, rho, u):
    g, h = _eq(C, p, rho, u)
    eu = fo3.edot(u)
    uu = np.sum(u * u, axis=1)[:, None]
    return g + fo3.W * rho[:, None] * fo3.CS2 * (eu * eu - fo3.CS2 * uu) / (2.0 * fo3.CS2 * fo3.CS2), h


_moments, _collide = fo3.moments, fo3.collide


def tau_arithmetic(C, prm):
    return C * prm.tau_l + (1.0 - C) * prm.tau_v


def velocity_without_density(g, h, prm):
    C, p, rho, u = _moments(g, h, prm)
    return C, p, rho, u * rho[:, None]


def collide_without_half(psi, psi_eq, tau):
    return psi - (psi - psi_eq) / tau[:, None]


_diagnostics = fo3.Oracle3D.diagnostics


def diagnostics_ke_doubled(self, g, h):
    d = _diagnostics(self, g, h)
    d["mean_ke"] *= 2.0
    return d


def diagnostics_ke_without_rho(self, g, h):
    d = _diagnostics(self, g, h)
    C, p, rho, u = fo3.moments(g, h, self.prm)
    d["mean_ke"] = float(0.5 * np.sum(u * u) / self.geo.N)
    return d


def _mixture_off():
    r = pins3d.mixture_viscosity_ratio()
    return not 1.0 < r < 1.2


_W = fo3.W.copy()

MUTATIONS = [
    ("face area -2V", "Geometry", GeometryTwoThirds, lambda: pins3d.laplacian_quadratic_error() > 1e-3),
    ("element lap mu doubled", "laplacian_mu", lapmu_doubled, lambda: pins3d.laplacian_quadratic_error() > 1e-3),
    ("no gradient averaging", "laplacian_C", lapC_no_average, lambda: pins3d.laplacian_quadratic_error() > 1e-3),
    ("wetting flux by the vertex rule", "wall_flux", wall_flux_trapezoid,
     lambda: pins3d.face_flux_quadrature_error() > 1e-6),
    ("missing incident wall faces", "laplacian_C", lapC_no_incident_wall_faces,
     lambda: pins3d.wall_linear_laplacian_error() > 1e-6),
    ("printed M10 sign", "rhs", rhs_printed_sign, lambda: pins3d.static_balance_drift() > 1e-8),
    ("dropped mobility term", "point_forces", forces_no_mobility, lambda: pins3d.force_moments_error() > 1e-8),
    ("eq:H pressure/mu term deleted", "point_forces", eqH_term_deleted,
     lambda: pins3d.first_step_composition_error_3d(0.5) > 0.05),
    ("eq:H mu grad C sign", "point_forces", eqH_mu_sign, lambda: pins3d.first_step_composition_error_3d(0.5) > 0.05),
    ("eq:H rho -> 1", "point_forces", eqH_rho_one, lambda: pins3d.first_step_composition_error_3d(0.5) > 0.05),
    ("Gamma quadratic coefficient doubled", "gamma", gamma_quadratic_doubled,
     lambda: pins3d.lattice_identities_error() > 1e-4),
    ("g_eq quadratic coefficient doubled", "equilibria", g_eq_quadratic_doubled,
     lambda: pins3d.lattice_identities_error() > 1e-4),
    ("arithmetic relaxation-time mixing", "relaxation_time", tau_arithmetic, _mixture_off),
    ("velocity moment without 1/rho", "moments", velocity_without_density, _mixture_off),
    ("collision rate 1/tau", "collide", collide_without_half, lambda: pins3d.shear_wave_viscosity_ratio() < 0.98),
    ("dropped dt^2 D term", "rhs", rhs_no_D, lambda: pins3d.static_balance_drift() > 1e-8),
    ("K sign", "rhs", rhs_K_sign, lambda: pins3d.static_balance_drift() > 1e-8),
    ("C transposed", "rhs", rhs_C_transposed, lambda: pins3d.static_balance_drift() > 1e-8),
    ("wetting flux sign", "wall_flux", wall_flux_flipped, lambda: pins3d.wall_linear_laplacian_error() > 1e-6),
    ("<T> doubled", "Oracle3D.diagnostics", diagnostics_ke_doubled, lambda: pins3d.diagnostics_error_3d() > 1e-6),
    ("<T> without rho", "Oracle3D.diagnostics", diagnostics_ke_without_rho,
     lambda: pins3d.diagnostics_error_3d() > 1e-6),
]


@pytest.mark.parametrize("name,attr,fn,caught", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pin_catches_planted_mistake_3d(monkeypatch, name, attr, fn, caught):
    owner, _, leaf = attr.rpartition(".")
    monkeypatch.setattr(getattr(fo3, owner) if owner else fo3, leaf, fn)
    assert caught(), f"no pin caught the planted mistake: {name}"


def test_wrong_d3q19_weight_is_caught(monkeypatch):
    w = _W.copy()
    w[7:] *= 1.01
    monkeypatch.setattr(fo3, "W", w)
    assert pins3d.lattice_identities_error() > 1e-4


def test_unmutated_3d_oracle_passes_the_same_predicates():
    assert not any(m[3]() for m in MUTATIONS)
