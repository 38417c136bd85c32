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
