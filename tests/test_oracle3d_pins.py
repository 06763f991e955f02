"""The 3-D CPU oracle (D3Q19 on P1 tetrahedra) pinned to what the paper and
mathematics fix (no GPU)."""
import pins3d


def test_tet_fem_matrices_match_bruteforce_quadrature():
    # eq:fem_matrices on one tetrahedron and on a jittered periodic 2 x 2 x 2 box
    assert pins3d.fem_bruteforce_error(pins3d.single_tet()) < 1e-9
    assert pins3d.fem_bruteforce_error(pins3d.small_box(n=2, nz=2)) < 1e-8


def test_tet_mass_matrix_closed_form():
    assert pins3d.single_tet_mass_error() < 1e-16


def test_tet_matrix_identities_and_wathen_bounds():
    for k, v in pins3d.identities_error().items():
        assert v < 1e-12, (k, v)


def test_d3q19_lattice_and_equilibrium_moments():
    assert pins3d.lattice_identities_error() < 1e-14


def test_static_interface_balance_3d():
    # Sec. II.C: the P0 force balances the streaming of a static profile exactly in 3-D too
    for seed in (3, 4):
        assert pins3d.static_balance_drift(seed) < 1e-14


def test_wall_face_flux_quadrature():
    assert pins3d.face_flux_quadrature_error() < 1e-13


def test_laplacians_on_quadratics():
    assert pins3d.laplacian_quadratic_error() < 1e-12


def test_wetting_flux_closes_linear_profile_at_walls():
    assert pins3d.wall_linear_laplacian_error() < 1e-12


def test_mass_conserved_3d():
    assert pins3d.mass_drift() < 1e-13


def test_no_slip_at_wall_nodes_3d():
    assert pins3d.wall_velocity_after_steps() < 1e-15


def test_force_moments_3d():
    assert pins3d.force_moments_error() < 1e-14


def test_viscosity_3d():
    assert 0.98 < pins3d.shear_wave_viscosity_ratio() < 1.08


def test_laplace_pressure_jump_3d():
    (q1, cont), (q2, _) = pins3d.laplace_jump(8.0, 1.0), pins3d.laplace_jump(8.0, 0.5)
    assert abs(cont - 1.0) < 0.01                  # the continuum integral is 2 sigma / R here
    assert abs((4.0 * q2 - q1) / 3.0 - 1.0) < 0.05  # Richardson-extrapolated discrete value
    assert (1.0 - q1) / (1.0 - q2) > 2.5            # converging at about second order


def test_first_step_composition_flux_of_eq_H_3d():
    # from rest with M = 0 the composition changes by dt^2/2 div[(C/rho)(grad p - mu grad C)],
    # which the h-scheme carries only through the C/(rho c_s^2)(grad p - mu grad C) term of eq:H
    e1, e2 = pins3d.first_step_composition_error_3d(1.0), pins3d.first_step_composition_error_3d(0.5)
    assert e2 < 0.01
    assert e1 / e2 > 3.0  # second order in h


def test_mixture_viscosity_3d():
    # a uniform mixture C = 1/2 shears with nu = c_s^2 tau dt at the relaxation time of
    # Sec. II.A (harmonic in C) and at density (rho_l + rho_v)/2
    r1, r2 = pins3d.mixture_viscosity_ratio(H=12), pins3d.mixture_viscosity_ratio(H=24, n_steps=600)
    assert r1 > r2 > 1.0                      # converging from above (1.10, 1.05; 1.02 at H = 48)
    assert abs(2.0 * r2 - r1 - 1.0) < 0.02    # first-order extrapolation to 1


def test_diagnostics_hand_count_3d():
    # mass, <T> and max |u> of a state whose velocities and density are set node by node
    assert pins3d.diagnostics_error_3d() < 1e-12
