"""The pins catch plausible mistakes planted in the oracle (CPU only).

Each planted mistake is one wrong expression at a PLANT(k) site of
oracle/cmlb_oracle.c or oracle/cmlb3_oracle.c (a comment at the site names
it), compiled in with -DORACLE_PLANT=k; the default build has none.  For each
k a copy of the oracle is built with that mistake, and the pin that should
catch it runs against that copy in a child process (the oracle module loads
the copy named by ORACLE_LIB) and must fail.  The 3D plants 21, 25 and 26
are caught by the pins that reduce the 3D oracle to the independently pinned
2D one on fields uniform along one axis.
"""
import concurrent.futures
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle_algebra.py", "tests/test_oracle_physics.py",
        "tests/test_oracle3.py", "tests/test_profile_pins.py"]

# planted mistake -> the pin that must catch it
PLANTS = {
    1: "test_laplace_law",                          # F_s without k_s
    2: "test_flow_equilibrium_raw_moments",         # first-order flow equilibria +psi u
    3: "test_translating_density_layer",            # factor 2 of the F_p sources dropped
    4: "test_sound_wave_damping",                   # B^-1 without its 1/2
    5: "test_transport_relations",                  # omega without 1/cs2
    6: "test_laplace_law",                          # gradient without 1/cs2
    7: "test_laplace_law",                          # curvature sign
    8: "test_couette_between_moving_walls",         # wall correction, incoming direction
    9: "test_tanh_sech2_steady_profiles",           # theta_c with 4/W
    10: "test_tanh_sech2_steady_profiles",          # sharpening flux dropped
    11: "test_F_against_definition",                # central moments about -u
    12: "test_advection_diffusion_mode",            # streamed against the direction
    13: "test_langmuir_special_cases",              # decimal logarithm
    14: "test_uniform_body_force",                  # velocity without the half force
    15: "test_marangoni_force_is_tangential",       # normal part of grad sigma kept
    16: "test_translating_density_layer",           # F_p from P^ instead of psi^
    17: "test_sound_wave_damping",                  # trace relaxed at the shear rate
    18: "test_layered_couette_viscosity_ratio",     # the two viscosities interchanged
    19: "test_laplace_law_abs_grad_reading",        # |grad phi|^2 kept in the |grad phi| reading
    20: "test_laplace_law_abs_grad_reading",        # its 1/(phi_a - phi_b) dropped
    21: "test_z_uniform_field_reduces_to_the_2d_oracle",  # 3D gradient without 1/cs2
    22: "test_axis_inverse_matches_dense_solve",    # 3D inverse, moving pair swapped
    23: "test_sound_wave_damping_3d",               # 3D trace at the shear rate
    24: "test_scalar_step_fourier_mode_exact3",     # streamed against z
    25: "test_z_uniform_field_reduces_to_the_2d_oracle",  # u u gamma source dropped
    26: "test_z_uniform_field_reduces_to_the_2d_oracle",  # corners left out of K
}


def _build_and_run(k, pin, tmp):
    import oracle
    path = os.path.join(tmp, f"liboracle_plant{k}.so")
    oracle.build(plant=k, out=path)
    env = dict(os.environ, ORACLE_LIB=path, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", *PINS, "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider", "-k", pin],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r


@pytest.fixture(scope="module")
def outcomes(tmp_path_factory):
    tmp = str(tmp_path_factory.mktemp("plants"))
    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
        futs = {k: ex.submit(_build_and_run, k, pin, tmp) for k, pin in PLANTS.items()}
        return {k: f.result() for k, f in futs.items()}


@pytest.mark.parametrize("k", sorted(PLANTS))
def test_pin_catches_planted_mistake(outcomes, k):
    r = outcomes[k]
    # pytest exits with 1 when a collected test failed; 5 (nothing collected)
    # or an error code would mean the pin did not run
    assert r.returncode == 1 and " failed" in r.stdout, (k, PLANTS[k], r.returncode,
                                                       r.stdout[-2000:], r.stderr[-2000:])


def test_unplanted_build_passes_the_pins(tmp_path):
    """The same build path with no plant passes the pins it runs above."""
    import oracle
    path = str(tmp_path / "liboracle_plant0.so")
    oracle.build(plant=0, out=path)
    env = dict(os.environ, ORACLE_LIB=path, OMP_NUM_THREADS="4")
    pins = " or ".join(sorted(set(PLANTS.values())))
    r = subprocess.run([sys.executable, "-m", "pytest", *PINS, "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider", "-k", pins],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:]
