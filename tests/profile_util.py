"""Interface profile of the surfactant, c_hat(theta), read off a field.

For the equilibrium profiles (Eqs. CACEeq and ISSeq) with phi_a = 1,
phi_b = 0: c = c_hat(theta) sech^2(2 zeta/W) and 4 phi (1 - phi) =
sech^2(2 zeta/W), so within an angular bin c_hat is the ratio of the bin's
sums of c and of 4 phi (1 - phi) over the interface band.  Sec. 4.1 gives the
closed form for the static drop, c_hat = (1 - exp(-D_s t/R^2) cos theta)/2."""
import numpy as np


def polar(nx, ny, xc, yc):
    x = np.arange(nx, dtype=np.float64)[None, :] - xc
    y = np.arange(ny, dtype=np.float64)[:, None] - yc
    return np.hypot(x, y), np.arctan2(y, x)


def interface_chat(phi, c, xc, yc, nbins=72, band=0.05, periodic_x=None):
    """(theta_centres, c_hat) over `nbins` equal angular bins around
    (xc, yc); nodes whose 4 phi (1 - phi) is below `band` are left out.
    `periodic_x`: box length for taking x offsets to the nearest image."""
    ny, nx = phi.shape
    x = np.arange(nx, dtype=np.float64)[None, :] - xc
    if periodic_x:
        x = (x + periodic_x / 2.0) % periodic_x - periodic_x / 2.0
    y = np.arange(ny, dtype=np.float64)[:, None] - yc
    th = np.broadcast_to(np.arctan2(y, x), phi.shape)
    w = 4.0 * phi * (1.0 - phi)
    m = w > band
    k = np.minimum(((th[m] + np.pi) / (2 * np.pi) * nbins).astype(int), nbins - 1)
    num = np.bincount(k, weights=c[m], minlength=nbins)
    den = np.bincount(k, weights=w[m], minlength=nbins)
    centres = -np.pi + (np.arange(nbins) + 0.5) * 2 * np.pi / nbins
    return centres, num / den


def chat_exact(theta, t_star, nbins=None):
    """Sec. 4.1 closed form; with `nbins`, cos theta is averaged over each
    bin (factor sin(h)/h, h = pi/nbins)."""
    f = 1.0
    if nbins:
        h = np.pi / nbins
        f = np.sin(h) / h
    return 0.5 * (1.0 - np.exp(-t_star) * f * np.cos(theta))


def taylor_deformation(phi, xc, yc, nray=720, level=0.5):
    """Taylor deformation D = (L - B)/(L + B) of the phi = `level` contour
    about (xc, yc): bilinear phi along `nray` rays (step 1/4), L and B the
    longest and shortest diameters (sums of opposite radii)."""
    ny, nx = phi.shape
    th = np.linspace(0.0, 2 * np.pi, nray, endpoint=False)
    rs = np.arange(0.0, min(nx, ny) / 2.0 - 2.0, 0.25)
    X = xc + np.cos(th)[:, None] * rs[None, :]
    Y = yc + np.sin(th)[:, None] * rs[None, :]
    x0 = np.floor(X).astype(int)
    y0 = np.floor(Y).astype(int)
    fx, fy = X - x0, Y - y0
    x0 %= nx
    x1 = (x0 + 1) % nx
    y0 = np.clip(y0, 0, ny - 1)
    y1 = np.clip(y0 + 1, 0, ny - 1)
    v = (phi[y0, x0] * (1 - fx) * (1 - fy) + phi[y0, x1] * fx * (1 - fy)
         + phi[y1, x0] * (1 - fx) * fy + phi[y1, x1] * fx * fy)
    r = np.empty(nray)
    for i in range(nray):
        k = int(np.argmax(v[i] < level))
        a, b = v[i, k - 1], v[i, k]
        r[i] = rs[k - 1] + (a - level) / (a - b) * (rs[k] - rs[k - 1])
    d = r[: nray // 2] + r[nray // 2:]
    L, B = d.max(), d.min()
    return float((L - B) / (L + B))


def stone_leal_D(Ca, beta, Pe, lam=1.0):
    """Sec. 4.3 small-deformation prediction D = 3 Ca b_r/(4 + Ca b_r)."""
    br = 1.25 * ((16 + 19 * lam) + 4 * beta * Pe / Ca) / (10 * (1 + lam) + 2 * beta * Pe / Ca)
    return 3 * Ca * br / (4 + Ca * br)


def fragments(phi, level=0.5):
    """Number of separate drops: connected regions of phi > `level` (nodes
    joined across edges), with the x direction periodic (a drop cut by the
    x seam counts once)."""
    from scipy import ndimage
    lab, n = ndimage.label(phi > level)
    if n < 2:
        return n
    root = list(range(n + 1))

    def find(i):
        while root[i] != i:
            i = root[i]
        return i

    for a, b in zip(lab[:, 0], lab[:, -1]):
        if a and b:
            root[find(b)] = find(a)
    return len({find(i) for i in range(1, n + 1)})
