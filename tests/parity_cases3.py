"""Named 3D (D3Q27) parity cases: builder() -> (params, fields), steps.
Sizes span several 64 x 4 collision columns with ragged x, y and z tails
(z: 2 to 40 planes, one to three column segments)."""
from paper_2504_09024_amd import workloads as W

CASES3 = {
    "static3": (lambda: W.static_drop3(n=40, R=11.0, D_s=0.05, center=(20.3, 19.7, 20.17)), 100),
    "prescribed3": (lambda: W.random_fields3(70, 20, 13, seed=4, flow="prescribed",
                                             bc_y="periodic", amp=1.0, M_phi=0.05), 60),
    "coupled3": (lambda: W.random_fields3(70, 22, 12, seed=3, amp=1.0, sigma0=2e-3, beta=0.3,
                                          u_wall=2e-2, M_phi=0.04, D_s=0.02), 60),
    "density3": (lambda: W.random_fields3(48, 16, 11, seed=5, amp=1.0, sigma0=1e-3, beta=0.2,
                                          rho_a=2.0, rho_b=1.0, nu_a=0.05, nu_b=0.1,
                                          omega_zeta=0.9, F_ext_x=1e-5, F_ext_y=-2e-5,
                                          F_ext_z=3e-5, bc_y="periodic"), 40),
    # the smallest grid: 4 x 4 x 1, every halo wraps or mirrors more than once
    "tiny3": (lambda: W.random_fields3(4, 4, 1, seed=7, amp=0.3, sigma0=1e-3, beta=0.2,
                                       u_wall=1e-2, M_phi=0.04, D_s=0.02), 10),
    # two planes: every z stencil wraps onto the same two planes
    "thin3": (lambda: W.random_fields3(40, 12, 2, seed=6, amp=1.0, sigma0=1e-3, beta=0.2,
                                       u_wall=1e-2, M_phi=0.04, D_s=0.02), 30),
    # Re = 1 shear drop (u ~ 1e-2, so the FP64 comparison is not at the
    # rounding floor of the velocity)
    "shear3": (lambda: W.shear_drop3(nx=96, ny=40, nz=24, R=8.0, Ca=0.3, E=0.2, c0=0.3,
                                     Re=1.0), 60),
}
