"""Plant plausible mistakes in the CPU oracle and check that a pin catches
each one (the pins would be worthless if a wrong oracle still passed them).
Every mistake is planted on the CPU, in the oracle module only."""
import numpy as np
import pytest

import pins
from oracle import felbm_oracle as fo

_rhs, _lapC, _lapmu, _forces = fo.rhs, fo.laplacian_C, fo.laplacian_mu, fo.element_forces
_wall, _collide, _wall_op, _equil = fo.wall_flux, fo.collide, fo.wall_operator, fo.equilibria


def rhs_printed_sign(mat, dt, psi_hat, Phi):
    # the sign printed in eq:galerkin_lbm: -(dt M10 - dt^2 K) Phi
    out = _rhs(mat, dt, psi_hat, np.zeros_like(Phi))
    for a in range(fo.Q):
        out[:, a] += -dt * (mat.M10 @ Phi[:, a]) + dt * dt * (mat.Ka[a] @ Phi[:, a])
    return out


def rhs_no_D(mat, dt, psi_hat, Phi):
    return np.stack([-dt * (mat.Ca[a] @ psi_hat[:, a]) + dt * (mat.M10 @ Phi[:, a]) + dt * dt * (mat.Ka[a] @ Phi[:, a])
                     for a in range(fo.Q)], 1)


def rhs_K_sign(mat, dt, psi_hat, Phi):
    return np.stack([-dt * (mat.Ca[a] @ psi_hat[:, a]) - dt * dt * (mat.Da[a] @ psi_hat[:, a])
                     + dt * (mat.M10 @ Phi[:, a]) - dt * dt * (mat.Ka[a] @ Phi[:, a]) for a in range(fo.Q)], 1)


def rhs_C_transposed(mat, dt, psi_hat, Phi):
    return np.stack([-dt * (mat.Ca[a].T @ psi_hat[:, a]) - dt * dt * (mat.Da[a] @ psi_hat[:, a])
                     + dt * (mat.M10 @ Phi[:, a]) + dt * dt * (mat.Ka[a] @ Phi[:, a]) for a in range(fo.Q)], 1)


def lapC_no_average(geo, C, gradC, bc):
    # inner element gradient only on every outer edge (no averaging with the neighbour)
    g2 = gradC.copy()
    saved = geo.edge_nbr.copy()
    geo.edge_nbr[:] = np.where(saved >= 0, np.arange(geo.NT)[:, None], saved)
    try:
        return _lapC(geo, C, g2, bc)
    finally:
        geo.edge_nbr[:] = saved


def wall_flux_flipped(C_a, C_b, r_a, r_b, length):
    return -_wall(C_a, C_b, r_a, r_b, length)


def lapC_no_incident_wall_edges(geo, C, gradC, bc):
    saved, saved_len = geo.wall_edges, geo.wall_len
    geo.wall_edges, geo.wall_len = saved[:0], saved_len[:0]
    try:
        return _lapC(geo, C, gradC, bc)
    finally:
        geo.wall_edges, geo.wall_len = saved, saved_len


def forces_e_not_e_minus_u(geo, prm, C, rho, u, mu, gradC, gradp, gradrho, lapmu):
    # Phi_h with e . X instead of (e - u) . X
    Pg, Ph = _forces(geo, prm, C, rho, u, mu, gradC, gradp, gradrho, lapmu)
    ub = u[geo.tri].mean(1)
    Cb, rhob, mub = C[geo.tri].mean(1), rho[geo.tri].mean(1), mu[geo.tri].mean(1)
    X = gradC - (Cb / (rhob * fo.CS2))[:, None] * (gradp - mub[:, None] * gradC)
    return Pg, Ph + (ub * X).sum(1)[:, None] * fo.gamma(ub)


def forces_no_mobility(geo, prm, C, rho, u, mu, gradC, gradp, gradrho, lapmu):
    return _forces(geo, prm, C, rho, u, mu, gradC, gradp, gradrho, 0 * lapmu)


def lapmu_wall_uses_own_gradient(geo, gradmu):
    saved_w = geo.edge_is_wall.copy(); saved_n = geo.edge_nbr.copy()
    geo.edge_is_wall[:] = False
    geo.edge_nbr[:] = np.where(saved_n >= 0, saved_n, np.arange(geo.NT)[:, None])
    try:
        return _lapmu(geo, gradmu)
    finally:
        geo.edge_is_wall[:] = saved_w; geo.edge_nbr[:] = saved_n


def collide_one_over_tau(psi, psi_eq, tau):
    return psi - (psi - psi_eq) / tau[:, None]


def no_wall_operator(geo, psi):
    return psi.copy()


def equilibria_wrong_weight(C, p, rho, u):
    g, h = _equil(C, p, rho, u)
    return g, h * (1.0 + 0.01 * (np.arange(fo.Q) == 5))


def nodal_matrices_factor(self):
    # 1/2 int d_r phi_i phi_j taken as (A/3) d_r N_i instead of (A/6) d_r N_i
    geo = self._geo
    tri, A, G = geo.tri, geo.area, geo.gradN
    I = np.repeat(tri, 3, axis=1).ravel()
    J = np.tile(tri, (1, 3)).ravel()
    li = np.repeat(np.arange(3), 3)
    import scipy.sparse as sp
    self.K1 = [sp.csr_matrix((((A[:, None] / 3.0) * G[:, li, r]).ravel(), (I, J)), shape=(geo.N, geo.N))
               for r in (0, 1)]
    self.K1a = [fo.E[a, 0] * self.K1[0] + fo.E[a, 1] * self.K1[1] for a in range(fo.Q)]
    return self.K1a


def nodal_average_unweighted(geo, elem_vec):
    acc = np.zeros((geo.N,) + elem_vec.shape[1:])
    cnt = np.zeros(geo.N)
    for l in range(3):
        np.add.at(acc, geo.tri[:, l], elem_vec)
        np.add.at(cnt, geo.tri[:, l], 1.0)
    return acc / cnt.reshape((-1,) + (1,) * (elem_vec.ndim - 1))


_point = fo.point_forces


def point_forces_no_mobility(prm, C, rho, u, mu, gradC, gradp, gradrho, lapmu):
    return _point(prm, C, rho, u, mu, gradC, gradp, gradrho, 0 * lapmu)


def _edot(u, X):
    return (fo.E[:, 0][None, :] - u[:, 0, None]) * X[:, 0, None] + (fo.E[:, 1][None, :] - u[:, 1, None]) * X[:, 1, None]


def _h_force(eq_h_term):
    """point_forces with the X vector of eq:H replaced by eq_h_term(C, rho, mu, gradC, gradp)."""
    def forces(prm, C, rho, u, mu, gradC, gradp, gradrho, lapmu):
        Pg, _ = _point(prm, C, rho, u, mu, gradC, gradp, gradrho, lapmu)
        Gu = fo.gamma(u)
        X = eq_h_term(C, rho, mu, gradC, gradp)
        return Pg, _edot(u, X) * Gu + prm.mobility * lapmu[:, None] * Gu
    return forces


eqH_term_deleted = _h_force(lambda C, rho, mu, gC, gp: gC)
eqH_mu_sign = _h_force(lambda C, rho, mu, gC, gp: gC - (C / (rho * fo.CS2))[:, None] * (gp + mu[:, None] * gC))
eqH_rho_one = _h_force(lambda C, rho, mu, gC, gp: gC - (C / fo.CS2)[:, None] * (gp - mu[:, None] * gC))

_gamma = fo.gamma


def gamma_quadratic_doubled(u):
    eu = u[..., 0, None] * fo.E[:, 0] + u[..., 1, None] * fo.E[:, 1]
    uu = (u[..., 0] * u[..., 0] + u[..., 1] * u[..., 1])[..., None]
    return fo.W * (1.0 + eu / fo.CS2 + (eu * eu - fo.CS2 * uu) / (fo.CS2 * fo.CS2))


def g_eq_quadratic_doubled(C, p, rho, u):
    g, h = _equil(C, p, rho, u)
    eu = u[:, 0, None] * fo.E[:, 0] + u[:, 1, None] * fo.E[:, 1]
    uu = (u[:, 0] * u[:, 0] + u[:, 1] * u[:, 1])[:, None]
    return g + fo.W * rho[:, None] * fo.CS2 * (eu * eu - fo.CS2 * uu) / (2.0 * fo.CS2 * fo.CS2), h


def laplacian_mu_doubled(geo, gradmu):
    return 2.0 * _lapmu(geo, gradmu)


_angle = fo.contact_angle


def contact_angle_supplement(mesh, C, level=0.5):
    th, h, b = _angle(mesh, C, level)
    return 180.0 - th, h, b


_diag = fo.Oracle.diagnostics


def band_ke_doubled(self, g, h, band=None):
    out = _diag(self, g, h, band)
    if "band_ke" in out:
        out["band_ke"] *= 2.0
    return out


_cwf = fo.collide_with_force


def collide_force_no_half_shift(psi, psi_eq, F, tau, dt):
    # the BGK term without the dt/2 F of the variable change (NC1)
    return psi - (psi - psi_eq) / (tau[:, None] + 0.5) + dt * F


_cforces = fo.Oracle._collision_forces


def collision_forces_no_c_star(self, C, rho, u, mu, gradC, gradp, gradrho, gradmu):
    out = _cforces(self, C, rho, u, mu, gradC, gradp, gradrho, gradmu)
    out["C_star"] = C
    return out


def collision_forces_full_at_walls(self, C, rho, u, mu, gradC, gradp, gradrho, gradmu):
    out = _cforces(self, C, rho, u, mu, gradC, gradp, gradrho, gradmu)
    out["F_g"], out["F_h"] = fo.point_forces(self.prm, C, rho, u, mu, out["gradC_n"], out["gradp_n"],
                                             out["gradrho_n"], out["lapmu_n"])
    return out


def init_without_half_force(self, C, u=None, p=None):
    N = self.geo.N
    u = np.zeros((N, 2)) if u is None else np.asarray(u)
    p = np.zeros(N) if p is None else np.asarray(p)
    g, h = fo.equilibria(np.asarray(C), p, fo.density(np.asarray(C), self.prm), u)
    return fo.wall_operator(self.geo, g), fo.wall_operator(self.geo, h)


_moments, _tau = fo.moments, fo.relaxation_time


def velocity_without_density(g, h, prm):
    C, p, rho, u = _moments(g, h, prm)
    return C, p, rho, u * rho[:, None]


def tau_arithmetic(C, prm):
    return C * prm.tau_l + (1.0 - C) * prm.tau_v


MUTATIONS = [
    ("printed M10 sign", "rhs", rhs_printed_sign, lambda: pins.static_balance_drift() > 1e-8),
    ("dropped D term", "rhs", rhs_no_D, lambda: pins.advection_error() > 0.05),
    ("K sign", "rhs", rhs_K_sign, lambda: pins.force_source_error() > 1e-5),
    ("C transposed", "rhs", rhs_C_transposed, lambda: pins.advection_error() > 0.05),
    ("no gradient averaging", "laplacian_C", lapC_no_average, lambda: pins.laplacian_quadratic_error() > 1e-4),
    ("wetting flux sign", "wall_flux", wall_flux_flipped, lambda: pins.wall_linear_laplacian_error() > 1e-4),
    ("wetting flux sign (wedge)", "wall_flux", wall_flux_flipped, lambda: pins.wall_flux_wedge_error(60.0) > 0.5),
    ("missing incident wall edges", "laplacian_C", lapC_no_incident_wall_edges,
     lambda: pins.wall_linear_laplacian_error() > 1e-4),
    ("(e - u) -> e in F_h", "element_forces", forces_e_not_e_minus_u, lambda: pins.force_moments_error() > 1e-8),
    ("dropped mobility term", "element_forces", forces_no_mobility, lambda: pins.force_moments_error() > 1e-8),
    ("nonzero wall flux of grad mu", "laplacian_mu", lapmu_wall_uses_own_gradient, lambda: pins.mass_drift() > 1e-10),
    ("collision rate 1/tau", "collide", collide_one_over_tau,
     lambda: not (0.98 < pins.shear_wave_viscosity_ratio(n_steps=300) < 1.08)),
    ("no wall operator", "wall_operator", no_wall_operator, lambda: pins.wall_velocity_after_step() > 1e-6),
    ("wrong equilibrium weight", "equilibria", equilibria_wrong_weight, lambda: pins.lattice_identities_error() > 1e-6),
    ("nodal force matrix factor", "Matrices.nodal_force_matrices", nodal_matrices_factor,
     lambda: pins.nodal_force_matrix_error() > 1e-3),
    ("unweighted nodal average", "nodal_average", nodal_average_unweighted, lambda: pins.nodal_average_error() > 1e-6),
    ("nodal forces without mobility", "point_forces", point_forces_no_mobility,
     lambda: pins.nodal_force_moments_error() > 1e-8),
    ("eq:H pressure/mu term deleted", "point_forces", eqH_term_deleted,
     lambda: pins.first_step_composition_error(0.5) > 0.05),
    ("eq:H mu grad C sign", "point_forces", eqH_mu_sign, lambda: pins.first_step_composition_error(0.5) > 0.05),
    ("eq:H rho -> 1", "point_forces", eqH_rho_one, lambda: pins.first_step_composition_error(0.5) > 0.05),
    ("Gamma quadratic doubled", "gamma", gamma_quadratic_doubled, lambda: pins.second_moment_error() > 1e-8),
    ("g_eq quadratic doubled", "equilibria", g_eq_quadratic_doubled, lambda: pins.second_moment_error() > 1e-8),
    ("element lap mu doubled", "laplacian_mu", laplacian_mu_doubled,
     lambda: pins.element_laplacian_quadratic_error() > 1e-3),
    ("contact angle pi - theta", "contact_angle", contact_angle_supplement,
     lambda: abs(pins.contact_angle_cap_errors(lambda m, C: fo.contact_angle(m, C)[0], 0.5)).max() > 0.5),
    ("band energy doubled", "Oracle.diagnostics", band_ke_doubled, lambda: pins.band_energy_error() > 1e-6),
    ("collision force without the dt/2 F shift", "collide_with_force", collide_force_no_half_shift,
     lambda: pins.collision_step_moment_error() > 1e-8),
    ("collision-step h equilibrium at C, not C*", "Oracle._collision_forces", collision_forces_no_c_star,
     lambda: pins.collision_step_moment_error() > 1e-8),
    ("collision-step force kept at wall nodes", "Oracle._collision_forces", collision_forces_full_at_walls,
     lambda: pins.collision_step_moment_error() > 1e-8),
    ("collision-step initial state without -dt/2 F", "Oracle.init_state", init_without_half_force,
     lambda: pins.first_step_composition_error(0.25, force_scheme="nodal_collide") > 0.5),
    ("velocity moment without 1/rho", "moments", velocity_without_density,
     lambda: pins.collision_conservation_error() > 1e-8),
    ("arithmetic relaxation-time mixing", "relaxation_time", tau_arithmetic,
     lambda: pins.relaxation_time_cases() > 1e-8),
]


@pytest.mark.parametrize("name,attr,fn,caught", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pin_catches_planted_mistake(monkeypatch, name, attr, fn, caught):
    owner, _, leaf = attr.rpartition(".")
    monkeypatch.setattr(getattr(fo, owner) if owner else fo, leaf, fn)
    assert caught(), f"no pin caught the planted mistake: {name}"


def test_unmutated_oracle_passes_the_same_predicates():
    assert not any(m[3]() for m in MUTATIONS)
