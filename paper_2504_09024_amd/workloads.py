"""Synthetic, seeded inputs for the coupled central-moment LB step.

This module holds only input construction: parameter sets and initial fields
built from the analytic set-ups of the paper's benchmarks (arXiv 2504.09024,
Sec. 4).  It contains none of the step's arithmetic, so both the GPU library's
tests and the CPU oracle's tests may draw their inputs from it.

Initial fields:
  * phase field: the tanh equilibrium profile, phi = phi_m + phi_o tanh(2 zeta/W)
    with zeta = R - |x - x_o| (Eq. CACEeq; Sec. 4.1 defines zeta);
  * surfactant: c = c_hat(theta) / cosh^2(2 zeta/W) (Eq. ISSeq; the static drop
    of Sec. 4.1 uses c_hat = (1 - cos theta)/2);
  * shear flow: u = U_o (2 y/H - 1) with y measured from the lower wall plane
    (Sec. 4.3).

Every function returns ``(params, fields)``: ``params`` is a dict keyed by the
library's parameter names, ``fields`` a dict of float64 arrays [ny][nx].
"""
from __future__ import annotations

import math

import numpy as np

CS2 = 1.0 / 3.0

BASE_PARAMS = dict(
    nx=64, ny=64, bc_y="periodic", flow="none",
    W=4.0, phi_a=1.0, phi_b=0.0, M_phi=0.1, D_s=0.01,
    rho_a=1.0, rho_b=1.0, nu_a=0.1, nu_b=0.1, omega_zeta=1.0,
    sigma0=0.0, beta=0.0, c_max=1.0,
    u_wall=0.0, F_ext_x=0.0, F_ext_y=0.0, vel_period_T=0.0,
)


def _sech2(s):
    """sech^2 s = 4 e^{-2|s|} / (1 + e^{-2|s|})^2, without overflow far from
    the interface."""
    e = np.exp(-2.0 * np.abs(s))
    return 4.0 * e / (1.0 + e) ** 2


def params(**kw) -> dict:
    p = dict(BASE_PARAMS)
    p.update(kw)
    return p


def drop_fields(nx, ny, xc, yc, R, W, c_hat=None, phi_a=1.0, phi_b=0.0, y_offset=0.0):
    """tanh drop (Eq. CACEeq) and sech^2 surfactant band (Eq. ISSeq).

    Node (i, j) sits at (i, j + y_offset).  ``c_hat`` is a callable of the
    polar angle theta (measured from +x), or a constant, or None (no
    surfactant)."""
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None] + y_offset
    dx = x - xc
    dy = y - yc
    r = np.sqrt(dx * dx + dy * dy)
    zeta = R - r
    phim = 0.5 * (phi_a + phi_b)
    phio = 0.5 * (phi_a - phi_b)
    phi = phim + phio * np.tanh(2.0 * zeta / W)
    theta = np.arctan2(dy, dx)
    if c_hat is None:
        ch = np.zeros_like(phi)
    elif callable(c_hat):
        ch = c_hat(theta)
    else:
        ch = np.full_like(phi, float(c_hat))
    c = ch * _sech2(2.0 * zeta / W)
    return np.ascontiguousarray(phi), np.ascontiguousarray(c)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def static_drop(n=128, R=32.0, W=4.0, D_s=0.01, M_phi=0.1, mode=1, center=None):
    """Static drop with a cos(mode*theta) surfactant gradient, u = 0
    (Sec. 4.1 set-up, scaled: 128x128 periodic, R = 32, W = 4, D_s = 0.01).
    c_hat = (1 - cos(mode theta))/2.  The centre defaults to the node
    (n/2, n/2)."""
    p = params(nx=n, ny=n, bc_y="periodic", flow="none", W=W, D_s=D_s, M_phi=M_phi)
    xc, yc = center if center is not None else (n / 2, n / 2)
    phi, c = drop_fields(n, n, xc, yc, R, W, lambda th: 0.5 * (1.0 - np.cos(mode * th)))
    return p, dict(phi=phi, c=c)


def advected_drop(Lo=512, R=None, W=4.0, D_s=0.1, M_phi=0.1, center=None):
    """Drop carried by a uniform flow along x on a periodic 2 Lo x Lo box
    (Sec. 4.2 set-up): R = Lo/4, c_hat = (1 - cos theta)/2, and U0 chosen so
    that the drop travels exactly Lo in T_D = R^2/D_s steps.  The velocity
    is a prescribed steady field (vel_period_T = 0)."""
    R = Lo / 4.0 if R is None else float(R)
    nx, ny = 2 * Lo, Lo
    T_D = R * R / D_s
    U0 = Lo / T_D
    p = params(nx=nx, ny=ny, bc_y="periodic", flow="prescribed", W=W, D_s=D_s, M_phi=M_phi,
               vel_period_T=0.0)
    xc, yc = center if center is not None else (Lo / 2.0, Lo / 2.0)
    phi, c = drop_fields(nx, ny, xc, yc, R, W, lambda th: 0.5 * (1.0 - np.cos(th)))
    return p, dict(phi=phi, c=c, ux=np.full((ny, nx), U0), uy=np.zeros((ny, nx)))


def vortex_drop(n=512, R=64.0, W=4.0, U0=0.02, T=20000.0, D_s=0.01, M_phi=0.1,
                center=None, c_hat=0.5):
    """Drop in a prescribed time-reversing single vortex on a periodic box.

    u =  U0 sin^2(pi x/L) sin(2 pi y/L) cos(pi t/T)
    v = -U0 sin^2(pi y/L) sin(2 pi x/L) cos(pi t/T)
    The shapes are passed as ux/uy; the library applies cos(pi t/T)."""
    if center is None:
        center = (n / 2, 0.75 * n)
    p = params(nx=n, ny=n, bc_y="periodic", flow="prescribed", W=W, D_s=D_s, M_phi=M_phi,
               vel_period_T=T)
    phi, c = drop_fields(n, n, center[0], center[1], R, W, c_hat)
    L = float(n)
    x = np.arange(n, dtype=np.float64)[None, :]
    y = np.arange(n, dtype=np.float64)[:, None]
    ux = U0 * np.sin(np.pi * x / L) ** 2 * np.sin(2 * np.pi * y / L)
    uy = -U0 * np.sin(np.pi * y / L) ** 2 * np.sin(2 * np.pi * x / L)
    ux = np.ascontiguousarray(np.broadcast_to(ux, (n, n)))
    uy = np.ascontiguousarray(np.broadcast_to(uy, (n, n)))
    return p, dict(phi=phi, c=c, ux=ux, uy=uy)


def shear_drop(nx=1024, ny=512, R=None, W=4.0, Ca=0.3, E=0.2, c0=0.3, Re=0.1, nu=0.1,
               Pe_s=1.0, Pe_star=0.5, rho=1.0, omega_zeta=1.0, c_max=1.0):
    """Surfactant-laden drop in simple shear between walls moving at +-U0
    (Sec. 4.3 set-up).  H = ny, R = H/8 unless given; drop at the channel
    centre; Re = gdot R^2/nu; Ca = mu gdot R/sigma0; Pe* = U0 W/M_phi (the
    paper uses 0.5); Pe_s = gdot R^2/D_s.  The velocity starts at the
    wall-driven linear profile u = U0 (2y/H - 1), y = j + 1/2."""
    H = float(ny)
    if R is None:
        R = H / 8.0
    gdot = Re * nu / (R * R)
    U0 = gdot * H / 2.0
    sigma0 = rho * nu * gdot * R / Ca
    M_phi = U0 * W / Pe_star
    D_s = gdot * R * R / Pe_s
    p = params(nx=nx, ny=ny, bc_y="walls", flow="coupled", W=W, M_phi=M_phi, D_s=D_s,
               rho_a=rho, rho_b=rho, nu_a=nu, nu_b=nu, omega_zeta=omega_zeta,
               sigma0=sigma0, beta=E, c_max=c_max, u_wall=U0)
    phi, c = drop_fields(nx, ny, nx / 2.0, H / 2.0, R, W, c0, y_offset=0.5)
    y = np.arange(ny, dtype=np.float64)[:, None] + 0.5
    ux = np.ascontiguousarray(np.broadcast_to(U0 * (2.0 * y / H - 1.0), (ny, nx)))
    uy = np.zeros((ny, nx))
    return p, dict(phi=phi, c=c, ux=ux, uy=uy)


def batched_shear_drops(n_sims=64, seed=2504, max_nodes=None):
    """64 independent coupled shear-drop runs with seeded sizes and parameters
    (numpy default_rng(seed)): ny uniform on {256, 320, ..., 512}; nx uniform
    on multiples of 64 in [ny, 1024]; R = ny/8; Ca ~ U[0.05, 0.6];
    E ~ U[0.1, 0.5]; c0 ~ U[0.1, 0.5]; Pe_s log-uniform on [0.5, 10];
    Re = 0.1, nu = 0.1, Pe* = 0.5.  ``max_nodes`` scales every grid down
    (keeping multiples of 16) for small test runs."""
    rng = np.random.default_rng(seed)
    sims = []
    for _ in range(n_sims):
        ny = int(rng.choice(np.arange(256, 513, 64)))
        nx_choices = np.arange(((ny + 63) // 64) * 64, 1025, 64)
        nx = int(rng.choice(nx_choices))
        Ca = float(rng.uniform(0.05, 0.6))
        E = float(rng.uniform(0.1, 0.5))
        c0 = float(rng.uniform(0.1, 0.5))
        Pe_s = float(math.exp(rng.uniform(math.log(0.5), math.log(10.0))))
        sims.append(dict(nx=nx, ny=ny, Ca=Ca, E=E, c0=c0, Pe_s=Pe_s))
    out = []
    for s in sims:
        nx, ny = s["nx"], s["ny"]
        if max_nodes is not None and nx * ny > max_nodes:
            f = math.sqrt(max_nodes / (nx * ny))
            nx = max(16, int(nx * f) // 16 * 16)
            ny = max(16, int(ny * f) // 16 * 16)
        out.append(shear_drop(nx=nx, ny=ny, Ca=s["Ca"], E=s["E"], c0=s["c0"], Pe_s=s["Pe_s"]))
    return out


def flat_interface(nx=64, ny=8, W=4.0, c_hat=0.0, M_phi=0.1, D_s=0.05):
    """Two flat tanh interfaces (normal along x) on a periodic box, with a
    uniform c_hat sech^2 band on each: the steady profiles of Eqs. CACEeq and
    ISSeq."""
    x = np.arange(nx, dtype=np.float64)[None, :]
    x1, x2 = nx / 4.0, 3.0 * nx / 4.0
    zeta = np.minimum(x - x1, x2 - x)
    phi = 0.5 + 0.5 * np.tanh(2.0 * zeta / W)
    c = c_hat * _sech2(2.0 * zeta / W)
    p = params(nx=nx, ny=ny, bc_y="periodic", flow="none", W=W, M_phi=M_phi, D_s=D_s)
    return p, dict(phi=np.ascontiguousarray(np.broadcast_to(phi, (ny, nx))),
                   c=np.ascontiguousarray(np.broadcast_to(c, (ny, nx))))


def _smooth_noise(rng, nx, ny, modes=4, periodic_y=True):
    """Sum of a few random low-wavenumber Fourier modes, unit RMS-ish."""
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    out = np.zeros((ny, nx))
    for _ in range(modes):
        kx = int(rng.integers(1, 4))
        ky = int(rng.integers(1, 4))
        ph = rng.uniform(0, 2 * np.pi, 2)
        ly = ny if periodic_y else 2 * ny
        out += np.cos(2 * np.pi * kx * x / nx + ph[0]) * np.cos(2 * np.pi * ky * y / ly + ph[1])
    return out / np.sqrt(modes)


def random_fields(nx, ny, seed=0, flow="coupled", bc_y="walls", amp=0.05, **kw):
    """Seeded smooth random fields for parity tests: an off-node drop with an
    angle-dependent surfactant load, plus low-wavenumber random perturbations
    of phi, c, u and P (smooth, so the case stays well conditioned)."""
    rng = np.random.default_rng(seed)
    p = params(nx=nx, ny=ny, bc_y=bc_y, flow=flow, **kw)
    R = min(nx, ny) / 4.0
    y_off = 0.5 if bc_y == "walls" else 0.0
    per = bc_y != "walls"
    phi, c = drop_fields(nx, ny, nx / 2.0 + 0.3, ny / 2.0 - 0.2, R, p["W"],
                         lambda th: 0.2 + 0.1 * np.cos(th) + 0.05 * np.sin(3 * th),
                         y_offset=y_off)
    phi = phi + amp * 0.1 * _smooth_noise(rng, nx, ny, periodic_y=per)
    c = c * (1.0 + amp * _smooth_noise(rng, nx, ny, periodic_y=per))
    ux = amp * 0.01 * _smooth_noise(rng, nx, ny, periodic_y=per)
    uy = amp * 0.01 * _smooth_noise(rng, nx, ny, periodic_y=per)
    P = CS2 + amp * 1e-3 * _smooth_noise(rng, nx, ny, periodic_y=per)
    return p, dict(phi=np.ascontiguousarray(phi), c=np.ascontiguousarray(c),
                   ux=np.ascontiguousarray(ux), uy=np.ascontiguousarray(uy),
                   P=np.ascontiguousarray(P))


def nodes(p) -> int:
    return int(p["nx"]) * int(p["ny"])


# ---------------------------------------------------------------------------
# Three-dimensional (D3Q27) inputs: the same analytic set-ups with a sphere
# (fields [nz][ny][nx], x fastest)
# ---------------------------------------------------------------------------

def params3(**kw) -> dict:
    p = params(**kw)
    p.setdefault("nz", 16)
    p.setdefault("F_ext_z", 0.0)
    return p


def drop_fields3(nx, ny, nz, xc, yc, zc, R, W, c_hat=None, phi_a=1.0, phi_b=0.0, y_offset=0.0):
    """tanh sphere (Eq. CACEeq with zeta = R - |x - x_o|) and sech^2
    surfactant band (Eq. ISSeq); node (i, j, k) sits at (i, j + y_offset, k).
    ``c_hat``: callable of (cos of the polar angle from +x), constant, or None."""
    x = np.arange(nx, dtype=np.float64)[None, None, :] - xc
    y = np.arange(ny, dtype=np.float64)[None, :, None] + y_offset - yc
    z = np.arange(nz, dtype=np.float64)[:, None, None] - zc
    r = np.sqrt(x * x + y * y + z * z)
    zeta = R - r
    phi = 0.5 * (phi_a + phi_b) + 0.5 * (phi_a - phi_b) * np.tanh(2.0 * zeta / W)
    if c_hat is None:
        ch = np.zeros_like(phi)
    elif callable(c_hat):
        ch = c_hat(np.where(r > 0, x / np.where(r > 0, r, 1.0), 0.0))
    else:
        ch = np.full_like(phi, float(c_hat))
    c = ch * _sech2(2.0 * zeta / W)
    return np.ascontiguousarray(phi), np.ascontiguousarray(c)


def static_drop3(n=64, R=16.0, W=4.0, D_s=0.05, M_phi=0.1, center=None):
    """Static sphere with c_hat = (1 - cos theta)/2 (theta from +x): the
    l = 1 surface mode of Sec. 4.1 in 3D, decaying as exp(-2 D_s t/R^2)."""
    p = params3(nx=n, ny=n, nz=n, bc_y="periodic", flow="none", W=W, D_s=D_s, M_phi=M_phi)
    xc, yc, zc = center if center is not None else (n / 2, n / 2, n / 2)
    phi, c = drop_fields3(n, n, n, xc, yc, zc, R, W, lambda ct: 0.5 * (1.0 - ct))
    return p, dict(phi=phi, c=c)


def _smooth_noise3(rng, nx, ny, nz, modes=4, periodic_y=True):
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    out = np.zeros((nz, ny, nx))
    ly = ny if periodic_y else 2 * ny
    for _ in range(modes):
        kx, ky, kz = (int(v) for v in rng.integers(1, 3, 3))
        ph = rng.uniform(0, 2 * np.pi, 3)
        out += (np.cos(2 * np.pi * kx * x / nx + ph[0]) * np.cos(2 * np.pi * ky * y / ly + ph[1])
                * np.cos(2 * np.pi * kz * z / nz + ph[2]))
    return out / np.sqrt(modes)


def random_fields3(nx, ny, nz, seed=0, flow="coupled", bc_y="walls", amp=0.05, **kw):
    """Seeded smooth 3D test fields: an off-node sphere with an
    angle-dependent surfactant load plus low-wavenumber perturbations of phi,
    c, u and P."""
    rng = np.random.default_rng(seed)
    p = params3(nx=nx, ny=ny, nz=nz, bc_y=bc_y, flow=flow, **kw)
    R = min(nx, ny, nz) / 3.0
    y_off = 0.5 if bc_y == "walls" else 0.0
    per = bc_y != "walls"
    phi, c = drop_fields3(nx, ny, nz, nx / 2.0 + 0.3, ny / 2.0 - 0.2, nz / 2.0 + 0.17, R, p["W"],
                          lambda ct: 0.2 + 0.1 * ct + 0.05 * ct * ct, y_offset=y_off)
    phi = phi + amp * 0.1 * _smooth_noise3(rng, nx, ny, nz, periodic_y=per)
    c = c * (1.0 + amp * _smooth_noise3(rng, nx, ny, nz, periodic_y=per))
    u = [amp * 0.01 * _smooth_noise3(rng, nx, ny, nz, periodic_y=per) for _ in range(3)]
    P = CS2 + amp * 1e-3 * _smooth_noise3(rng, nx, ny, nz, periodic_y=per)
    return p, dict(phi=np.ascontiguousarray(phi), c=np.ascontiguousarray(c),
                   ux=np.ascontiguousarray(u[0]), uy=np.ascontiguousarray(u[1]),
                   uz=np.ascontiguousarray(u[2]), P=np.ascontiguousarray(P))


def shear_drop3(nx=256, ny=128, nz=128, R=32.0, W=4.0, Ca=0.3, E=0.2, c0=0.3, Re=0.1, nu=0.1,
                Pe_s=1.0, Pe_star=0.5, rho=1.0, omega_zeta=1.0, c_max=1.0):
    """3D surfactant-laden drop in simple shear between walls at y = -1/2 and
    ny - 1/2 moving at -+U0 along x, periodic in x and z: the Sec. 4.3
    set-up with a sphere (parameters defined as in shear_drop)."""
    H = float(ny)
    gdot = Re * nu / (R * R)
    U0 = gdot * H / 2.0
    p = params3(nx=nx, ny=ny, nz=nz, bc_y="walls", flow="coupled", W=W,
                M_phi=U0 * W / Pe_star, D_s=gdot * R * R / Pe_s, rho_a=rho, rho_b=rho,
                nu_a=nu, nu_b=nu, omega_zeta=omega_zeta, sigma0=rho * nu * gdot * R / Ca,
                beta=E, c_max=c_max, u_wall=U0)
    phi, c = drop_fields3(nx, ny, nz, nx / 2.0, H / 2.0, nz / 2.0, R, W, c0, y_offset=0.5)
    y = np.arange(ny, dtype=np.float64)[None, :, None] + 0.5
    ux = np.ascontiguousarray(np.broadcast_to(U0 * (2.0 * y / H - 1.0), (nz, ny, nx)))
    return p, dict(phi=phi, c=c, ux=ux, uy=np.zeros((nz, ny, nx)), uz=np.zeros((nz, ny, nx)))
