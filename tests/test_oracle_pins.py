"""The CPU oracle pinned to what the paper and mathematics fix (no GPU)."""
import pytest

import pins


def test_fem_matrices_match_bruteforce_quadrature():
    # eq:fem_matrices on the four-element mesh and on a jittered periodic mesh
    assert pins.fem_bruteforce_error() < 1e-9
    assert pins.fem_bruteforce_error(pins.small_mesh(nx=6, ny=4)) < 1e-9


def test_mass_matrix_closed_form_four_elements():
    assert pins.m11_golden_error() < 1e-15


def test_matrix_identities():
    errs = pins.identities_error()
    for k, v in errs.items():
        assert v < 1e-13, (k, v)


def test_d2q9_lattice_and_equilibrium_moments():
    assert pins.lattice_identities_error() < 1e-14


def test_collision_conserves_and_fixes_equilibrium():
    assert pins.collision_conservation_error() < 1e-14


def test_relaxation_time_special_cases():
    assert pins.relaxation_time_cases() < 1e-14


def test_static_interface_balance():
    # Sec. II.C: the P0 force exactly balances the streaming of a static profile
    for seed in (3, 4):
        assert pins.static_balance_drift(seed) < 1e-14


def test_streaming_advects_along_characteristics():
    assert pins.advection_error() < 0.02


def test_streaming_force_source():
    assert pins.force_source_error() < 1e-8


def test_patch_laplacian_exact_on_quadratics():
    assert pins.laplacian_quadratic_error() < 1e-12


def test_patch_laplacian_second_order():
    assert 3.5 < pins.laplacian_cosine_ratio() < 4.5


def test_wetting_flux_closes_linear_profile_at_wall():
    assert pins.wall_linear_laplacian_error() < 1e-12


@pytest.mark.parametrize("theta", [45.0, 60.0, 120.0, 135.0])
def test_wetting_flux_matches_young_wedge(theta):
    # eq. bc2 + Young's relation: the planar tanh interface at angle theta
    assert pins.wall_flux_wedge_error(theta) < 0.01


def test_wall_flux_quadrature():
    assert pins.simpson_wall_flux_error() < 1e-13


def test_surface_tension_of_tanh_profile():
    assert pins.surface_tension_integral() < 0.02


def test_flat_interface_chemical_potential_converges():
    e1, e2 = pins.flat_interface_mu(1.0), pins.flat_interface_mu(0.5)
    assert e2 < 0.1
    assert 2.5 < e1 / e2 < 5.0


@pytest.mark.parametrize("R", [16.0, 24.0])
def test_laplace_pressure_jump(R):
    f1, f2 = pins.laplace_jump(R, 1.0), pins.laplace_jump(R, 0.5)
    extrap = (4.0 * f2 - f1) / 3.0          # second-order Richardson extrapolation in h
    assert abs(extrap - 1.0) < 0.02
    assert abs(f2 - 1.0) < 0.05


def test_mass_conserved_with_wetting_wall():
    assert pins.mass_drift() < 1e-13


def test_no_slip_at_wall_nodes():
    assert pins.wall_velocity_after_step() < 1e-15


def test_mesh_with_holes():
    area, closure, drift, wall_u = pins.channel_mesh_pins()
    assert area < 1e-14
    assert closure < 1e-13
    assert drift < 1e-13
    assert wall_u < 1e-15


def test_pcg_matches_dense_solve():
    assert pins.pcg_dense_error() < 1e-12


def test_force_moments():
    assert pins.force_moments_error() < 1e-14


def test_viscosity_from_relaxation_time():
    assert 0.98 < pins.shear_wave_viscosity_ratio() < 1.08


def test_complex_step_tangent_matches_fd():
    assert pins.complex_step_vs_fd() < 1e-6


def test_nodal_force_matrix_matches_bruteforce():
    assert pins.nodal_force_matrix_error() < 1e-8


def test_nodal_average_is_patch_centroid():
    assert pins.nodal_average_error() < 1e-12


def test_nodal_forces_do_not_balance_static_interface():
    # the mixed scheme keeps this state to rounding (test_static_interface_balance);
    # the nodal one moves it, which is the mechanism behind the parasitic-current table
    assert pins.nodal_static_drift() > 1e-4


def test_nodal_force_moments():
    assert pins.nodal_force_moments_error() < 1e-14


def test_nodal_scheme_conserves_mass():
    assert pins.nodal_mass_drift() < 1e-12
