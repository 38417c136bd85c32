"""Paper-scale runs on the GPU against closed forms and invariants (sizes
beyond the oracle's reach).

* Sec. 4.1: static drop, 512 x 512, R = 128, W = 4, D_s in {0.05, 0.1, 0.2}
  (one batched launch per step), read at t* = D_s t/R^2 up to 1 and beyond:
  the interface profile c_hat(theta) against (1 - exp(-t*) cos theta)/2.
* Sec. 4.2: the same drop on a 1024 x 512 box carried by a uniform flow
  over Lo = 512 columns in T_D = R^2/D_s steps: profile about the shifted
  centre, and phi against the initial drop moved by 512 columns.
* 3D: the steady Taylor deformation of a clean drop in shear against
  35/32 Ca, and its growth with confinement and with surfactant; a sphere's
  l = 1 surfactant mode carried across a periodic box (Sec. 4.2 in 3D).
* Single vortex (512 x 512, R = 64, U0 = 0.02, T = 20000): after the full
  reversal period the drop returns; one step deep in the run against the
  oracle at full size.
* Density and viscosity ratios: two-layer Couette flow (mu_a/mu_b = 4) with
  a continuous shear stress.
"""
import math

import numpy as np
import pytest

from paper_2504_09024_amd import workloads as W
from parity_util import gpu_ctx
from profile_util import chat_exact, interface_chat

pytestmark = pytest.mark.gpu

NB = 72


def _profile_err(f, xc, yc, t_star, periodic_x=None):
    th, ch = interface_chat(f["phi"], f["c"], xc, yc, nbins=NB, periodic_x=periodic_x)
    return float(np.abs(ch - chat_exact(th, t_star, nbins=NB)).max())


def test_static_drop_paper_scale_fp64(gpu_lib):
    """Max |c_hat - closed form| over 72 bins stays below 3e-3 (t=0 read-out
    error 1e-3 included) for every D_s at every checkpoint up to t* = 4."""
    n, R = 512, 128.0
    Ds = (0.05, 0.1, 0.2)
    cases = [W.static_drop(n=n, R=R, D_s=d, M_phi=0.1) for d in Ds]
    ctx = gpu_ctx([c[0] for c in cases], [c[1] for c in cases], "fp64")
    chunk = 40960  # T_D/4 for D_s = 0.1
    worst = {}
    for k in range(1, 9):
        ctx.step(chunk)
        for i, d in enumerate(Ds):
            t_star = d * k * chunk / R ** 2
            e = _profile_err(ctx.read_fields(i), n / 2, n / 2, t_star)
            worst[(d, t_star)] = e
            print(f"D_s={d} t*={t_star:.3f} max|dc_hat|={e:.2e}", flush=True)
    assert ctx.fault_flags(0) == 0
    for key, e in worst.items():
        assert e < 3e-3, (key, e)
    ctx.close()


def test_advected_drop_paper_scale_fp64(gpu_lib):
    """After t* = 1 the drop has moved 512 columns: profile error about the
    shifted centre below 3e-3, and phi within 2e-2 (relative L2) of the
    initial drop shifted by 512 columns."""
    p, fl = W.advected_drop(Lo=512, D_s=0.1)
    R = 128.0
    T_D = int(R * R / p["D_s"])
    ctx = gpu_ctx(p, fl, "fp64")
    ctx.step(T_D)
    f = ctx.read_fields(0)
    e = _profile_err(f, 256.0 + 512.0, 256.0, 1.0, periodic_x=1024)
    moved = np.roll(fl["phi"], 512, axis=1)
    dphi = float(np.linalg.norm(f["phi"] - moved) / np.linalg.norm(moved))
    print(f"advected: max|dc_hat|={e:.2e}  phi vs shifted initial {dphi:.2e}")
    assert e < 3e-3, e
    assert dphi < 2e-2, dphi
    s0 = (fl["phi"].sum(), fl["c"].sum())
    s1 = ctx.inventory(0)
    assert abs(s1[0] - s0[0]) / s0[0] < 1e-12
    assert abs(s1[1] - s0[1]) / s0[1] < 1e-12
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_vortex_full_period(gpu_lib, prec):
    """512 x 512 single vortex, T = 20000: phi at t = T returns to phi(0)
    within 5e-2 relative L2; Sigma phi and Sigma c conserved."""
    p, fl = W.vortex_drop()
    ctx = gpu_ctx(p, fl, prec)
    s0 = ctx.inventory(0)
    ctx.step(20000)
    f = ctx.read_fields(0)
    s1 = ctx.inventory(0)
    ret = float(np.linalg.norm(f["phi"] - fl["phi"]) / np.linalg.norm(fl["phi"]))
    drift = [abs(a - b) / abs(b) for a, b in zip(s1, s0)]
    print(f"{prec} vortex: |phi(T)-phi(0)|/|phi(0)| = {ret:.3e}, drift {drift}")
    assert ret < 5e-2, ret
    assert max(drift) < (1e-12 if prec == "fp64" else 1e-5), drift
    ctx.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 1e-6)])
def test_vortex_one_step_deep_in_the_run(oracle_mod, gpu_lib, prec, tol):
    """Full-size vortex: after 3000 GPU steps, one more step from the GPU's
    own populations through the oracle matches the GPU's step (max
    population difference relative to the largest population).  Checks the
    per-step arithmetic far into the run, where multi-step comparisons are
    limited by the problem's conditioning."""
    p, fl = W.vortex_drop(center=(256.3, 383.6))
    ctx = gpu_ctx(p, fl, prec)
    ctx.step(3000)
    f, h, _ = ctx.get_populations(0)
    o = oracle_mod.OracleSim.from_populations(oracle_mod.make_params(**p), f, h, None, t=3000,
                                              ux_shape=fl["ux"], uy_shape=fl["uy"])
    ctx.step(1)
    assert o.run(1) == 0
    gf, gh, _ = ctx.get_populations(0)
    for a, b in ((gf, o.f), (gh, o.h)):
        d = np.abs(a - b).max() / np.abs(b).max()
        print(prec, f"one-step max rel diff {d:.2e}")
        assert d <= tol, d
    ctx.close()


# Sec. 4.3 table (clean and contaminated D x 1e-2 at Re = 0.1)
PAPER_TABLE = {0.01: (1.60, 1.89), 0.02: (3.19, 3.72), 0.03: (4.77, 5.55),
               0.04: (6.35, 7.36), 0.05: (7.93, 9.17)}


def test_shear_drop_deformation_paper_scale(gpu_lib):
    """Sec. 4.3 set-up: 768 x 256 channel, R = 32, Re = 0.1, Ca = 0.01 ...
    0.05, clean (beta = 0, no surfactant) and contaminated (beta = 0.25,
    c0 = 0.3, D_s from Pe_s = 1) at the paper's Pe* = U0 W/M_phi = 0.5, and
    clean at Pe* = 1 and 2; all twenty drops in one launch, FP32, 4e5 steps
    (gdot t = 3.9).

    At Pe* = 0.5 the clean D is steady and linear in Ca, surfactant raises
    it, and both lie at 0.80-0.82 of the paper's table (band 0.78-0.85).
    The factor is the Cahn-Hilliard-type mobility, which the paper names as
    the parameter these results are sensitive to: with U0 the wall speed and
    W = 4, lowering M_phi raises D monotonically toward the table (D/Ca =
    1.28, 1.39, 1.59 at Pe* = 0.5, 1, 2 for Ca = 0.02; 1.20 at Pe* = 0.125),
    and at Pe* = 2 the mean of D/D_table over the five Ca lies within 6% of
    one.  A thinner interface acts the same way (W = 3: 1.47; R = 64 with
    W = 4: 1.37), a wider one the other way (W = 6 and 8: 1.21).  At Pe* = 2
    phi over- and undershoots by 1.4% and D still grows between gdot t = 3
    and 4 and falls off with Ca, so that mobility is not used for the
    steady checks."""
    from profile_util import stone_leal_D, taylor_deformation
    Cas = sorted(PAPER_TABLE)
    cases = [W.shear_drop(nx=768, ny=256, R=32.0, Ca=ca, E=0.0, c0=0.0) for ca in Cas]
    cases += [W.shear_drop(nx=768, ny=256, R=32.0, Ca=ca, E=0.25, c0=0.3, Pe_s=1.0)
              for ca in Cas]
    for pes in (1.0, 2.0):
        cases += [W.shear_drop(nx=768, ny=256, R=32.0, Ca=ca, E=0.0, c0=0.0, Pe_star=pes)
                  for ca in Cas]
    ctx = gpu_ctx([c[0] for c in cases], [c[1] for c in cases], "fp32")
    D = {}
    for steps in (300000, 100000):
        ctx.step(steps)
        D[steps] = [taylor_deformation(ctx.read_fields(i)["phi"], 384.0, 127.5)
                    for i in range(len(cases))]
    assert all(ctx.fault_flags(i) == 0 for i in range(len(cases)))
    ctx.close()
    d3, d4 = D[300000], D[100000]
    Pe = 0.1 * 0.1 / cases[5][0]["D_s"]
    print("Ca   D_clean  D_cont  (x1e-2; table clean/cont; Stone-Leal clean/cont); "
          "clean D at Pe* = 1, 2")
    for i, ca in enumerate(Cas):
        print(f"{ca:.2f} {100 * d4[i]:7.3f} {100 * d4[5 + i]:7.3f}   {PAPER_TABLE[ca][0]:.2f}/"
              f"{PAPER_TABLE[ca][1]:.2f}   {100 * stone_leal_D(ca, 0, Pe):.3f}/"
              f"{100 * stone_leal_D(ca, 0.25, Pe):.3f}   {100 * d4[10 + i]:7.3f} "
              f"{100 * d4[15 + i]:7.3f}", flush=True)
    for i, ca in enumerate(Cas):
        assert abs(d4[i] - d3[i]) < 0.02 * d4[i], (ca, d3[i], d4[i])  # clean: steady
        assert d4[5 + i] > d4[i], ca                                  # surfactant raises D
        for j, k in ((i, 0), (5 + i, 1)):                             # 0.80-0.82 of the table
            assert 0.78 < d4[j] / (PAPER_TABLE[ca][k] * 1e-2) < 0.85, (ca, k, d4[j])
        assert d4[i] < d4[10 + i] < d4[15 + i], ca                     # lower mobility, larger D
    slope = [d4[i] / ca for i, ca in enumerate(Cas)]
    assert max(slope) / min(slope) < 1.05, slope                     # linear regime
    low_m = np.mean([d4[15 + i] / (PAPER_TABLE[ca][0] * 1e-2) for i, ca in enumerate(Cas)])
    assert abs(low_m - 1.0) < 0.06, low_m


def test_taylor_deformation_3d(gpu_lib):
    """3D (D3Q27) clean drop in simple shear at small Ca, Re = 0.1: the steady
    Taylor deformation D of the phi = 1/2 contour in the shear plane.
    Taylor's small-deformation result for equal viscosities is
    D = (19 + 16)/(16 + 16) Ca = 35/32 Ca; the W = 4 interface carries an
    effective tension of ~0.94 sigma0 (the 3D Laplace test), so the
    unconfined expectation is D/Ca ~ 1.17.  With walls at 2R/H = 0.2 and
    periodic images (8R apart in x, 5R in z) the measured D/Ca must lie
    within [1.0, 1.2] of that; D is steady (gdot t = 3 against 4), linear in
    Ca (0.1 against 0.05), grows with confinement (2R/H = 0.4), and grows
    with surfactant (beta = 0.25, c0 = 0.3, Pe_s = 1), as in Sec. 4.3."""
    from profile_util import taylor_deformation

    def run(R, Ca, nx, ny, nz, E=0.0, c0=0.0):
        p, fl = W.shear_drop3(nx=nx, ny=ny, nz=nz, R=R, Ca=Ca, E=E, c0=c0, Re=0.1)
        gdot = 0.1 * 0.1 / (R * R)
        ctx = cmlb_ctx3(p, fl)
        out, done = [], 0
        for g in (3.0, 4.0):
            n = int(round(g / gdot))
            ctx.step(n - done)
            done = n
            out.append(taylor_deformation(ctx.read_fields(0)["phi"][nz // 2], nx / 2.0,
                                          ny / 2.0 - 0.5))
        assert ctx.fault_flags(0) == 0
        ctx.close()
        print(f"3D Taylor R={R} Ca={Ca} 2R/H={2 * R / ny:.2f} beta={E}: D={out[1]:.4f} "
              f"D/Ca={out[1] / Ca:.3f} (35/32 = {35 / 32:.3f})", flush=True)
        return out

    d1 = run(16.0, 0.1, 128, 160, 80)
    d2 = run(16.0, 0.05, 128, 160, 80)
    for d in (d1, d2):
        assert abs(d[1] - d[0]) < 0.01 * d[1]                      # steady
    assert abs(d1[1] / (2 * d2[1]) - 1) < 0.05                     # linear in Ca
    ratio = (d1[1] / 0.1) / (35 / 32 / 0.94)
    assert 1.0 < ratio < 1.2, ratio
    dw = run(12.0, 0.1, 96, 120, 64)
    dn = run(12.0, 0.1, 96, 60, 64)
    assert dn[1] > 1.05 * dw[1]                                     # confinement raises D
    ds = run(12.0, 0.1, 96, 120, 64, E=0.25, c0=0.3)
    assert ds[1] > 1.05 * dw[1]                                     # surfactant raises D


def cmlb_ctx3(p, fl):
    from paper_2504_09024_amd import cmlb
    ctx = cmlb.Context3(p, "fp32")
    ctx.init_fields(0, fl["phi"], fl["c"], fl["ux"], fl["uy"], fl["uz"])
    return ctx


def test_advected_sphere_3d(gpu_lib):
    """Sec. 4.2 in 3D: a sphere (R = 16) with the l = 1 surfactant mode
    carried once across a periodic 96 x 64 x 64 box by a uniform flow
    (U = 0.02 along x, 4800 steps), FP32.  Back at its start, phi matches
    the initial sphere (relative L2 below 2e-2, the diffuse interface's
    numerical dispersion) and the mode has decayed as exp(-2 D_s t/R^2)
    (within 5%), as it does at rest: the surface diffusion is Galilean
    invariant."""
    from paper_2504_09024_amd import cmlb
    n, R, D, U = 64, 16.0, 0.05, 0.02
    nx = 96
    steps = int(round(nx / U))
    p = W.params3(nx=nx, ny=n, nz=n, bc_y="periodic", flow="prescribed", W=4.0, D_s=D,
                  M_phi=0.1)
    xc, yc, zc = nx / 2.0 + 0.3, n / 2.0 - 0.2, n / 2.0 + 0.1
    phi0, c0 = W.drop_fields3(nx, n, n, xc, yc, zc, R, 4.0, lambda ct: 0.5 * (1.0 - ct))
    ux = np.full((n, n, nx), U)
    zero = np.zeros((n, n, nx))
    ctx = cmlb.Context3(p, "fp32")
    ctx.init_fields(0, phi0, c0, ux, zero, zero)
    x = np.arange(nx)[None, None, :] - xc
    y = np.arange(n)[None, :, None] - yc
    z = np.arange(n)[:, None, None] - zc
    ct = x / np.sqrt(x * x + y * y + z * z)

    def amp(cc):
        return (cc * ct).sum() / cc.sum()

    a0 = amp(ctx.read_fields(0)["c"])
    ctx.step(steps)
    f = ctx.read_fields(0)
    assert ctx.fault_flags(0) == 0
    ctx.close()
    decay = -math.log(amp(f["c"]) / a0)
    expected = 2 * D * steps / R ** 2
    err = float(np.linalg.norm(f["phi"] - phi0) / np.linalg.norm(phi0))
    print(f"advected sphere: decay {decay:.4f} expected {expected:.4f}; phi rel L2 {err:.2e}")
    assert abs(decay / expected - 1) < 0.05
    assert err < 2e-2


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-3), ("fp32", 4e-3)])
def test_layered_couette_viscosity_ratio(gpu_lib, prec, tol):
    """Two fluid layers between the moving walls on the GPU path: fluid a
    (rho 2, nu 0.1) below a flat interface at mid-height, fluid b (rho 1,
    nu 0.05) above, 64 x 128, walls at +-U.  In the steady state the shear
    stress is the same at every height: the bulk slopes stand in the ratio
    mu_b/mu_a = 1/4 (mu = rho nu), and the stress is 2U / sum_j 1/mu(phi_j)
    with rho and nu linear in phi (App. D).  FP32 settles into a steady
    state within 9e-4 of U of the FP64 one (slope ratio 0.25072): over the
    3e5 steps a per-step FP32 rounding that repeats at every node of this
    steady flow is integrated over the viscous time H^2/nu."""
    nx, ny, U = 64, 128, 1e-3
    ra, rb, na, nb = 2.0, 1.0, 0.1, 0.05
    p = W.params(nx=nx, ny=ny, flow="coupled", bc_y="walls", u_wall=U, sigma0=0.0, beta=0.0,
                 M_phi=0.02, D_s=0.01, rho_a=ra, rho_b=rb, nu_a=na, nu_b=nb)
    y = np.arange(ny)[:, None] + 0.5 + 0 * np.arange(nx)[None, :]
    phi = 0.5 + 0.5 * np.tanh(2 * (ny / 2 - y) / 4.0)
    z = np.zeros_like(phi)
    ctx = gpu_ctx(p, dict(phi=phi, c=z, P=np.full_like(phi, rb / 3.0)), prec)
    ctx.step(300000)  # >= 9 decay times H^2/(pi^2 nu) of the slowest mode
    f = ctx.read_fields(0)
    ctx.close()
    u, ph = f["ux"].mean(axis=1), f["phi"].mean(axis=1)
    assert np.abs(f["ux"] - u[:, None]).max() < 1e-9 * U
    yy = np.arange(ny) + 0.5
    la = (yy > 4) & (yy < ny / 2 - 12)
    lb = (yy > ny / 2 + 12) & (yy < ny - 4)
    sa = np.polyfit(yy[la], u[la], 1)[0]
    sb = np.polyfit(yy[lb], u[lb], 1)[0]
    mu = (rb + ph * (ra - rb)) * (nb + ph * (na - nb))
    tau = 2 * U / np.sum(1.0 / mu)
    print(f"{prec}: slope ratio {sa / sb:.6f} (1/4), stress {ra * na * sa:.6e} vs {tau:.6e}",
          flush=True)
    assert abs((sa / sb) / (rb * nb / (ra * na)) - 1) < tol
    assert abs(ra * na * sa / tau - 1) < 3e-3


BREAKUP_BETAS = (0.0, 0.25, 0.5)


@pytest.mark.parametrize("re,t_end,prec", [(1.0, 25.0, "fp32"), (1.0, 25.0, "fp64"),
                                           (4.0, 12.0, "fp32")])
def test_drop_breakup_in_shear(gpu_lib, re, t_end, prec):
    """Sec. 4.3 break-up runs: 768 x 256 channel, R = 32, Ca = 0.35, clean
    (beta = 0) and surfactant-laden (beta = 0.25, 0.5 with c0 = 0.3, Pe_s =
    1, as in the deformation runs), all three in one launch, to t* = gdot t
    of 25 at Re = 1 and 12 at Re = 4.  The paper shows these runs only as
    pictures, so nothing here is compared with numbers of its (parity
    unpinned); what is checked is what its text states: every drop breaks;
    at Re = 1 into two, the surfactant-laden drops first and the more
    sensitive (larger beta) one earliest; at Re = 4 into several drops.
    Drops are counted every quarter unit of t*.  Measured at Re = 1: first
    break at t* = 18.0 (beta = 0.5), 20.25 (0.25), 24.25 (clean), the same in
    FP32 and FP64; at Re = 4 at t* = 11-11.25 into 7-9 drops.  Also: no
    fault, and the inventories: FP64 to rounding, FP32 to 5e-4 in phi
    (1.7e-4 measured over the 2.6e5 steps at Re = 1: storage rounding that
    repeats at the slowly changing nodes) and c."""
    from profile_util import fragments
    cases = [W.shear_drop(nx=768, ny=256, R=32.0, Ca=0.35, E=b, c0=0.3 if b else 0.0, Re=re)
             for b in BREAKUP_BETAS]
    ctx = gpu_ctx([c[0] for c in cases], [c[1] for c in cases], prec)
    inv0 = np.array([[c[1]["phi"].sum(), c[1]["c"].sum()] for c in cases])
    gdot = re * 0.1 / 32.0 ** 2
    broke = {}
    done = 0
    for k in range(1, int(round(t_end * 4)) + 1):
        n = int(round(k * 0.25 / gdot))
        ctx.step(n - done)
        done = n
        for i, b in enumerate(BREAKUP_BETAS):
            if b not in broke and fragments(ctx.read_fields(i)["phi"]) > 1:
                broke[b] = k * 0.25
    last = [fragments(ctx.read_fields(i)["phi"]) for i in range(3)]
    inv = np.array(ctx.inventories(0, 3))
    faults = [ctx.fault_flags(i) for i in range(3)]
    ctx.close()
    drift = np.abs(inv - inv0) / np.maximum(inv0, 1e-300)
    print(f"Re={re} {prec}: first break at t* {broke}; drops at t*={t_end}: {last}; "
          f"drift {drift.tolist()}", flush=True)
    assert faults == [0, 0, 0]
    assert np.all(drift <= (1e-11 if prec == "fp64" else 5e-4)), drift
    assert set(broke) == set(BREAKUP_BETAS), broke
    if re == 1.0:
        assert last == [2, 2, 2], last
        assert broke[0.5] < broke[0.25] < broke[0.0], broke
    else:
        assert min(last) >= 3, last


def test_contaminated_drop_drift_and_its_limit(gpu_lib):
    """The contaminated Sec. 4.3 drop (Ca = 0.01, beta = 0.25, c0 = 0.3,
    Pe_s = 1, FP32) at the paper's Pe* = 0.5 does not settle: phi over- and
    undershoots by 2-3e-3 near the interface, so the equilibrium profile
    c_hat 4 phi (1 - phi) is negative there and the confining flux moves
    surfactant out of the bulk (bulk c turns negative, total c stays) onto
    the interface, where c_hat keeps rising until c reaches c_max = 1 and
    the Langmuir fault stops the run (measured: c_hat averages 0.86 on the
    interface after 1e6 steps; the fault comes between 1.4e6 and 1.5e6
    steps; asserted: between 1.2e6 and 2e6).  With four times the mobility
    (Pe* = 0.125) phi stays within 1e-5 of [0, 1] and the same drop holds
    c_hat at 0.289 from 1e5 steps to the end: the drift comes from the
    boundedness error of phi, not from the surfactant scheme."""
    from paper_2504_09024_amd import cmlb
    cases = [W.shear_drop(nx=768, ny=256, R=32.0, Ca=0.01, E=0.25, c0=0.3, Pe_s=1.0,
                          Pe_star=pes) for pes in (0.5, 0.125)]
    ctx = gpu_ctx([c[0] for c in cases], [c[1] for c in cases], "fp32")

    def chat_mean(fl):
        w = 4 * fl["phi"] * (1 - fl["phi"])
        band = w > 0.5
        return float((fl["c"][band] / w[band]).mean())

    hist = {0: [], 1: []}
    fault_at = None
    for k in range(1, 21):
        ctx.step(100000)
        try:
            fls = [ctx.read_fields(i) for i in range(2)]
        except cmlb.CmlbError as e:
            assert e.code == cmlb.ERANGE
            fault_at = k * 100000
            break
        for i, fl in enumerate(fls):
            hist[i].append((chat_mean(fl), fl["phi"].min(), fl["phi"].max(), fl["c"].min()))
    flags = [ctx.fault_flags(i) for i in range(2)]
    ctx.close()
    print("Pe* = 0.5 c_hat:", [round(h[0], 3) for h in hist[0]], "fault at", fault_at, flush=True)
    print("Pe* = 0.125 c_hat:", [round(h[0], 4) for h in hist[1]], flush=True)
    assert fault_at is not None and 1200000 < fault_at <= 2000000, fault_at
    assert flags[0] & 2 and flags[1] == 0, flags
    a = hist[0]
    assert min(h[1] for h in a[2:]) < -1e-3 and max(h[2] for h in a[2:]) > 1 + 1e-3
    assert a[9][0] > a[0][0] + 0.4                      # c_hat climbs by 1e6 steps
    assert a[-1][3] < -5e-3                             # bulk c negative
    b = hist[1]
    assert all(-1e-5 < h[1] and h[2] < 1 + 1e-5 for h in b)
    assert max(h[0] for h in b) - min(h[0] for h in b) < 2e-3
