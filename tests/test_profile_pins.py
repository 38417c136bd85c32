"""CPU pins of the interface-profile read-out used by the paper-scale GPU
validations, and of the oracle's surface diffusion against the Sec. 4.1
closed form c_hat(theta, t) = (1 - exp(-D_s t/R^2) cos theta)/2."""
import numpy as np

from paper_2504_09024_amd import workloads as W
from profile_util import chat_exact, interface_chat


def test_readout_of_initial_profile():
    """The read-out returns the imposed (1 - cos theta)/2 at t = 0."""
    p, fl = W.static_drop(n=512, R=128.0, D_s=0.1)
    th, ch = interface_chat(fl["phi"], fl["c"], 256.0, 256.0)
    err = np.abs(ch - chat_exact(th, 0.0, nbins=72)).max()
    assert err < 2e-3, err


def test_readout_of_shifted_drop_across_the_periodic_seam():
    """A drop rolled across the x seam of a periodic box reads the same."""
    p, fl = W.advected_drop(Lo=128)
    phi, c = (np.roll(fl[k], 166, axis=1) for k in ("phi", "c"))
    th, ch = interface_chat(phi, c, 64.0 + 166.0, 64.0, periodic_x=256)
    # R = 32: nodal sampling of 72 bins leaves ~6e-3
    assert np.abs(ch - chat_exact(th, 0.0, nbins=72)).max() < 1e-2


def test_oracle_profile_follows_closed_form(oracle_mod):
    """64x64, R = 16, D_s = 0.1: after T_D/4 = 640 steps the read-out profile
    matches exp(-1/4) decay of the cos theta mode to 1.5e-2 (diffuse-interface
    corrections are O((W/R)^2) at this small radius)."""
    n, R, D = 64, 16.0, 0.1
    p, fl = W.static_drop(n=n, R=R, D_s=D, M_phi=0.1, center=(32.0, 32.0))
    s = oracle_mod.OracleSim(oracle_mod.make_params(**p), fl["phi"], fl["c"])
    steps = int(R * R / D / 4)
    assert s.run(steps) == 0
    f = s.fields()
    th, ch = interface_chat(f["phi"], f["c"], 32.0, 32.0, nbins=24)
    err = np.abs(ch - chat_exact(th, D * steps / R ** 2, nbins=24)).max()
    # a plausible mistake (no diffusion, or twice the rate) is >= 0.09 off
    assert err < 1.5e-2, err


def test_taylor_deformation_of_exact_ellipses():
    """D of a diffuse ellipse (tanh profile across its boundary, W = 4) with
    semi-axes a, b at several inclinations is (a - b)/(a + b) to 1e-3."""
    from profile_util import taylor_deformation
    ny, nx = 256, 768
    x = np.arange(nx)[None, :] - 384.0
    y = np.arange(ny)[:, None] - 127.5
    for a, b, ang in ((40.0, 25.0, 0.5), (34.0, 30.0, 0.8), (32.0, 32.0, 0.0)):
        xr = x * np.cos(ang) + y * np.sin(ang)
        yr = -x * np.sin(ang) + y * np.cos(ang)
        rr = np.sqrt((xr / a) ** 2 + (yr / b) ** 2)
        phi = 0.5 + 0.5 * np.tanh(2 * (1 - rr) * np.sqrt(a * b) / 4.0)
        assert abs(taylor_deformation(phi, 384.0, 127.5) - (a - b) / (a + b)) < 1e-3


def test_stone_leal_reduces_to_its_clean_limit():
    """beta = 0: b_r = 5(16 + 19 lam)/(40 (1 + lam)), independent of Pe."""
    from profile_util import stone_leal_D
    for Ca in (0.01, 0.05):
        br = 5 * 35 / 80
        assert abs(stone_leal_D(Ca, 0.0, 7.0) - 3 * Ca * br / (4 + Ca * br)) < 1e-15
    assert stone_leal_D(0.01, 0.25, 1.0) > stone_leal_D(0.01, 0.0, 1.0)


def test_fragment_count():
    """Drops are counted once each, also when the periodic x seam cuts one;
    a thin neck still joins, a gap of one node separates."""
    from profile_util import fragments
    phi = np.zeros((40, 60))
    assert fragments(phi) == 0
    phi[5:10, 5:15] = 1.0
    assert fragments(phi) == 1
    phi[20:30, 0:4] = 1.0
    phi[22:28, 55:60] = 1.0          # one drop across the seam
    assert fragments(phi) == 2
    phi[7, 15:30] = 1.0              # a one-node neck joins a third blob
    phi[5:10, 30:40] = 1.0
    assert fragments(phi) == 2
    phi[7, 22] = 0.0                 # neck cut: the blob is separate
    assert fragments(phi) == 3
    phi[33, 33] = 0.9                # diagonal neighbours are not joined
    phi[34, 34] = 0.9
    assert fragments(phi) == 5
