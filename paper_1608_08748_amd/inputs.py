"""Seeded synthetic initial conditions (primitive variables only).

This module holds no arithmetic of the numerical method: it only draws and
shapes initial data.  Both the HIP path and the CPU oracle consume its output.

Every generator returns a float64 array ``W`` of shape (10, nz, ny, nx) with the
primitive fields, x fastest in memory:

    rho, vx, vy, vz, p, bx_f, by_f, bz_f, x_h2, x_hp

where ``bx_f[k, j, i]`` is B_x on the lower x face (i-1/2, j, k) of the cell
(and likewise for y and z), ``x_h2`` is the H2 mass fraction and ``x_hp`` the H+ mass fraction (zero
unless a generator is asked for ionised gas).  Units are
Heaviside-Lorentz (B^2/2 is the magnetic pressure), the box is the periodic
unit cube with cubic cells of edge h = 1/nx.

The turbulence recipe stands in for the paper's chemo-MHD turbulence run
(Sec. 4.3: periodic box, uniform density, random velocity, uniform field along
one axis, molecular-hydrogen chemistry): velocity is a Gaussian random field
with shell spectrum E(k) ~ k^-2 over integer wavenumbers 1 <= |k| <= 8,
normalised to a given rms Mach number; the mean field is along x with a given
plasma beta = 2 p0 / B0^2; pressure is isothermal p = p0 rho / rho0.
"""
import numpy as np

PRIM = ("rho", "vx", "vy", "vz", "p", "bx_f", "by_f", "bz_f", "x_h2", "x_hp")


def _alloc(shape):
    nz, ny, nx = shape
    return np.zeros((10, nz, ny, nx), dtype=np.float64)


def uniform(shape, rho=1.0, v=(0.0, 0.0, 0.0), p=1.0, B=(0.0, 0.0, 0.0), x_h2=1e-3):
    W = _alloc(shape)
    W[0] = rho
    W[1], W[2], W[3] = v
    W[4] = p
    W[5], W[6], W[7] = B
    W[8] = x_h2
    return W


def white_noise(shape, seed=1, sigma=0.1, rho=1.0, p=1.0, B=(0.1, 0.0, 0.0), x_h2=1e-3):
    """Uniform gas with independent Gaussian velocity per cell and component."""
    rng = np.random.default_rng(seed)
    W = uniform(shape, rho=rho, p=p, B=B, x_h2=x_h2)
    W[1:4] = rng.normal(0.0, sigma, size=(3,) + tuple(shape))
    return W


def c1(n=32, seed=1):
    """32^3 box, rho = 1, p = 1, B = (0.1, 0, 0), white-noise velocity sigma 0.1, x_H2 = 1e-3."""
    return white_noise((n, n, n), seed=seed, sigma=0.1, B=(0.1, 0.0, 0.0), x_h2=1e-3)


def _spectral_field(rng, shape, kmin=1, kmax=8, slope=-2.0, dtype=np.float64):
    """Real Gaussian random field with shell spectrum E(k) ~ k^slope on integer
    shells kmin <= |k| <= kmax, unit variance."""
    import scipy.fft as sfft
    nz, ny, nx = shape
    rdt = np.float32 if dtype == np.float32 else np.float64
    cdt = np.complex64 if dtype == np.float32 else np.complex128
    kz = np.fft.fftfreq(nz, 1.0 / nz).astype(rdt)[:, None, None]
    ky = np.fft.fftfreq(ny, 1.0 / ny).astype(rdt)[None, :, None]
    kx = np.arange(nx // 2 + 1, dtype=rdt)[None, None, :]
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    shell = np.rint(kk)
    mask = (shell >= kmin) & (shell <= kmax) & (kk > 0)
    del shell
    # E(k) ~ k^slope in a shell of area ~k^2 means |a_k|^2 ~ k^(slope-2)
    amp = np.zeros_like(kk)
    amp[mask] = kk[mask] ** ((slope - 2.0) / 2.0)
    del kk, mask
    spec = np.empty(amp.shape, dtype=cdt)
    spec.real = rng.standard_normal(amp.shape, dtype=rdt)
    spec.imag = rng.standard_normal(amp.shape, dtype=rdt)
    spec *= amp
    del amp
    f = sfft.irfftn(spec, s=(nz, ny, nx), axes=(0, 1, 2), workers=-1, overwrite_x=True)
    del spec
    f -= f.mean(dtype=np.float64)
    s = float(np.sqrt(np.mean(np.square(f, dtype=np.float64))))
    if s > 0:
        f /= s
    return f


def turbulence(n, seed, mach, beta, x_h2, lognormal_sigma=None, rho0=1.0, p0=1.0, gamma=5.0 / 3.0, log=None):
    """Supersonic MHD turbulence start: GRF velocity (k^-2, k = 1..8) at rms
    Mach ``mach``, mean field B0 = sqrt(2 p0 / beta) along x, isothermal
    pressure p = p0 rho / rho0, optional lognormal density of width sigma.
    ``n``: cells per axis of a cube, or a shape (nz, ny, nx) (thin boxes keep
    the wavenumbers their axes can hold).
    ``log``: optional callable given a progress string after each field."""
    shape = (n, n, n) if np.isscalar(n) else tuple(int(x) for x in n)
    rng = np.random.default_rng(seed)
    # boxes of 512^3 and more draw their random fields in single precision
    dt = np.float32 if int(np.prod(shape)) >= 512 ** 3 else np.float64
    W = _alloc(shape)
    if lognormal_sigma is None:
        W[0] = rho0
    else:
        g = _spectral_field(rng, shape, dtype=dt)
        s = float(lognormal_sigma)
        W[0] = np.exp(s * g - 0.5 * s * s)
        del g
        W[0] *= rho0 / W[0].mean()
        if log:
            log("density done")
    ms = 0.0
    for d in range(3):
        W[1 + d] = _spectral_field(rng, shape, dtype=dt)
        ms += float(np.mean(np.square(W[1 + d])))
        if log:
            log("velocity %d done" % d)
    cs0 = np.sqrt(gamma * p0 / rho0)
    W[1:4] *= mach * cs0 / np.sqrt(ms)
    np.multiply(W[0], p0 / rho0, out=W[4])
    W[5] = np.sqrt(2.0 * p0 / beta)
    W[8] = x_h2
    return W


def c2(n=256, seed=2):
    """256^3, rho = 1, rms Mach 5, beta = 1, x_H2 = 1e-3."""
    return turbulence(n, seed, mach=5.0, beta=1.0, x_h2=1e-3)


def c3(n=512, seed=3):
    """512^3, rms Mach 5, beta = 0.3, x_H2 = 1e-3."""
    return turbulence(n, seed, mach=5.0, beta=0.3, x_h2=1e-3)


def c4(n=1024, seed=4, log=None):
    """1024^3, lognormal density (sigma 1), rms Mach 10, beta = 0.1, x_H2 = 1e-2."""
    return turbulence(n, seed, mach=10.0, beta=0.1, x_h2=1e-2, lognormal_sigma=1.0, log=log)


def serving_requests(count=256, seed=5, sizes=(32, 48, 64, 96, 128), rate=None):
    """Request list for the serving workload: size, Mach, beta, x_H2, seed and
    (if ``rate`` is given, in requests/s) Poisson arrival times."""
    rng = np.random.default_rng(seed)
    reqs = []
    t = 0.0
    for r in range(count):
        n = int(rng.choice(sizes))
        mach = float(rng.uniform(1.0, 10.0))
        beta = float(rng.uniform(0.1, 10.0))
        xh2 = float(10.0 ** rng.uniform(-4.0, -1.0))
        if rate is not None:
            t += float(rng.exponential(1.0 / rate))
        reqs.append(dict(id=r, n=n, mach=mach, beta=beta, x_h2=xh2, seed=int(rng.integers(1 << 31)), t_arrive=t))
    return reqs


def request_state(req):
    return turbulence(req["n"], req["seed"], mach=req["mach"], beta=req["beta"], x_h2=req["x_h2"])


# ---------------------------------------------------------------- test problems


def riemann_1d(n, left, right, gamma_free_B=(0.0,), x0=0.5, x_h2=0.0):
    """Periodic double Riemann problem on an n x 1 x 1 box: the left state fills
    [0, x0), the right state [x0, 1).  States are dicts with rho, p, vx, vy, vz,
    by, bz and the common bx (normal field)."""
    W = _alloc((1, 1, n))
    x = (np.arange(n) + 0.5) / n
    L = x < x0
    for s, m in ((left, L), (right, ~L)):
        W[0, 0, 0, m] = s["rho"]
        W[1, 0, 0, m] = s.get("vx", 0.0)
        W[2, 0, 0, m] = s.get("vy", 0.0)
        W[3, 0, 0, m] = s.get("vz", 0.0)
        W[4, 0, 0, m] = s["p"]
        W[6, 0, 0, m] = s.get("by", 0.0)
        W[7, 0, 0, m] = s.get("bz", 0.0)
    W[5] = left.get("bx", 0.0)
    W[8] = x_h2
    return W


def sod(n):
    return riemann_1d(n, dict(rho=1.0, p=1.0), dict(rho=0.125, p=0.1))


def barmin(n):
    """MHD shock tube of Sec. 3.1 (field already in Heaviside-Lorentz units, gamma 1.4)."""
    left = dict(rho=0.18405, p=0.3541, vx=3.8964, vy=0.5361, vz=2.4866, by=2.394, bz=1.197, bx=4.0)
    right = dict(rho=0.1, p=0.1, vx=-5.5, vy=0.0, vz=0.0, by=2.0, bz=1.0, bx=4.0)
    return riemann_1d(n, left, right)


def advected_density_wave(n, amp=0.2, v=1.0, p=1.0):
    """rho = 1 + amp sin(2 pi x) (exact cell averages), uniform velocity and pressure, B = 0."""
    W = _alloc((1, 1, n))
    xl = np.arange(n) / n
    xr = (np.arange(n) + 1) / n
    W[0, 0, 0] = 1.0 + amp * (np.cos(2 * np.pi * xl) - np.cos(2 * np.pi * xr)) / (2 * np.pi / n)
    W[1] = v
    W[4] = p
    return W


def alfven_wave(n, amp=0.1, bx=1.0, rho=1.0, p=0.1):
    """Circularly polarised Alfven wave along x (exact nonlinear solution):
    B_perp = amp (sin, cos)(2 pi x), v_perp = -B_perp / sqrt(rho), travelling
    in +x at speed bx / sqrt(rho).  Exact cell averages."""
    W = _alloc((1, 1, n))
    xl = np.arange(n) / n
    xr = (np.arange(n) + 1) / n
    k = 2 * np.pi
    s_avg = (np.cos(k * xl) - np.cos(k * xr)) / (k / n)
    c_avg = (np.sin(k * xr) - np.sin(k * xl)) / (k / n)
    W[0] = rho
    W[4] = p
    W[5] = bx
    W[6, 0, 0] = amp * s_avg
    W[7, 0, 0] = amp * c_avg
    W[2, 0, 0] = -amp * s_avg / np.sqrt(rho)
    W[3, 0, 0] = -amp * c_avg / np.sqrt(rho)
    return W


def orszag_tang(n):
    """Orszag-Tang vortex of Sec. 3.2 on an n x n x 1 box; the face field is the
    discrete curl of A_z = B0 (cos(4 pi x) / (4 pi) + cos(2 pi y) / (2 pi))."""
    W = _alloc((1, n, n))
    h = 1.0 / n
    B0 = 1.0 / np.sqrt(4 * np.pi)
    xc = (np.arange(n) + 0.5) * h
    xf = np.arange(n + 1) * h

    def Az(x, y):
        return B0 * (np.cos(4 * np.pi * x) / (4 * np.pi) + np.cos(2 * np.pi * y) / (2 * np.pi))

    X, Y = np.meshgrid(xc, xc, indexing="xy")
    W[0, 0] = 25.0 / (36.0 * np.pi)
    W[4, 0] = 5.0 / (12.0 * np.pi)
    W[1, 0] = -np.sin(2 * np.pi * Y)
    W[2, 0] = np.sin(2 * np.pi * X)
    # corners (x_{i-1/2}, y_{j-1/2}) for i, j in 0..n
    XF, YF = np.meshgrid(xf, xf, indexing="xy")
    A = Az(XF, YF)   # shape (n+1 [y], n+1 [x])
    # bx on face (i-1/2, j) = (A(i-1/2, j+1/2) - A(i-1/2, j-1/2)) / h
    W[5, 0] = (A[1:, :-1] - A[:-1, :-1]) / h
    # by on face (i, j-1/2) = -(A(i+1/2, j-1/2) - A(i-1/2, j-1/2)) / h
    W[6, 0] = -(A[:-1, 1:] - A[:-1, :-1]) / h
    return W


def divfree_random(shape, seed, amp=0.1, B0=(0.1, 0.0, 0.0)):
    """Face field = uniform B0 + discrete curl of a random edge vector potential
    (discretely divergence free).  Returns the three face arrays."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    h = 1.0 / nx
    Ax, Ay, Az = (rng.normal(0.0, amp * h, size=shape) for _ in range(3))
    # A_x on edge (i, j-1/2, k-1/2), A_y on (i-1/2, j, k-1/2), A_z on (i-1/2, j-1/2, k)
    def up(a, axis):
        return np.roll(a, -1, axis=axis)
    # axis 0 = z, 1 = y, 2 = x
    bx = B0[0] + ((up(Az, 1) - Az) - (up(Ay, 0) - Ay)) / h
    by = B0[1] + ((up(Ax, 0) - Ax) - (up(Az, 2) - Az)) / h
    bz = B0[2] + ((up(Ay, 2) - Ay) - (up(Ax, 1) - Ax)) / h
    return bx, by, bz
