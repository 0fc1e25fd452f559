"""Seeded synthetic inputs (density fields and right-hand sides).

This module holds no arithmetic of the solver: it only draws random numbers
and evaluates closed-form density profiles and band-limited random fields,
so that the GPU path and the CPU oracle are fed identical arrays.  Shapes
follow the paper's test problems (top-hat density of eq. VDINSE.rho.hat;
tanh interfaces as in the Rayleigh-Taylor set-up of Sec. 4.3; a jet-like
radial profile as in the swirling-jet case of Sec. 4.3) at the grid sizes of
the workloads below.

Every field is float64, C order, x the last (contiguous) axis.
"""
import numpy as np

TWO_PI = 2.0 * np.pi


def _rng(*key):
    return np.random.default_rng(np.random.SeedSequence([int(k) for k in key]))


def grid_1d(n, length=TWO_PI):
    return length * np.arange(n) / n


def band_limited(shape, band, seed, keep_mean=False, tag=0):
    """Real periodic random field with Gaussian Fourier coefficients on
    |kappa_d| <= band along every axis (no Nyquist content), unit RMS.
    The k = 0 coefficient is dropped unless ``keep_mean``."""
    rng = _rng(seed, tag, len(shape), *shape)
    hshape = tuple(shape[:-1]) + (shape[-1] // 2 + 1,)
    coef = rng.standard_normal(hshape) + 1j * rng.standard_normal(hshape)
    mask = np.ones(hshape, dtype=bool)
    for d, n in enumerate(shape):
        idx = np.fft.fftfreq(n, d=1.0 / n) if d < len(shape) - 1 else np.arange(hshape[-1])
        sel = np.abs(idx) <= band
        shp = [1] * len(shape)
        shp[d] = hshape[d]
        mask &= sel.reshape(shp)
    coef[~mask] = 0.0
    if not keep_mean:
        coef[(0,) * len(shape)] = 0.0
    else:
        coef[(0,) * len(shape)] = rng.standard_normal() * np.sqrt(2.0)
    u = np.fft.irfftn(coef, s=shape, axes=tuple(range(len(shape))))
    rms = np.sqrt(np.mean(u * u))
    return np.ascontiguousarray(u / rms)


# ------------------------------------------------------------- 1D top-hat

def tophat_1d(n=256, r=3.0, x1=np.pi / 2, x2=3 * np.pi / 2, d=0.05):
    """rho(x) = 1 + (r-1)/2 [tanh((x-x1)/d) - tanh((x-x2)/d)] on [0, 2 pi)."""
    x = grid_1d(n)
    return 1.0 + 0.5 * (r - 1.0) * (np.tanh((x - x1) / d) - np.tanh((x - x2) / d))


def rhs_1d(n=256, band=64, seed=0):
    """f = sum_{k=1..band} alpha_k cos kx + beta_k sin kx, alpha, beta ~ N(0,1)."""
    rng = _rng(seed, 1, n)
    x = grid_1d(n)
    a = rng.standard_normal(band)
    b = rng.standard_normal(band)
    k = np.arange(1, band + 1)
    return np.cos(np.outer(x, k)) @ a + np.sin(np.outer(x, k)) @ b


def c1_inputs(seed=0, n=256):
    return {"rho": tophat_1d(n), "f": rhs_1d(n, band=n // 4, seed=seed),
            "lengths": (TWO_PI,)}


# ----------------------------------------------------- 3D jet-like density

def jet_density(n, rj, width=0.05, radius=0.5):
    """rho = 1 + (rj-1)/2 (1 - tanh((r_perp - radius)/width)), axis along x.

    r_perp is the distance to the line (y, z) = (pi, pi).  Shape (n, n, n).
    """
    x = grid_1d(n)
    zz, yy = np.meshgrid(x, x, indexing="ij")
    rp = np.sqrt((yy - np.pi) ** 2 + (zz - np.pi) ** 2)
    plane = 1.0 + 0.5 * (rj - 1.0) * (1.0 - np.tanh((rp - radius) / width))
    return np.ascontiguousarray(np.broadcast_to(plane[:, :, None], (n, n, n)))


def c3_inputs(rj=3.0, n=256, seed=0, with_g=False):
    out = {"rho": jet_density(n, rj),
           "f": band_limited((n, n, n), n // 4, seed, tag=3),
           "lengths": (TWO_PI,) * 3}
    if with_g:
        out["g"] = np.stack([band_limited((n, n, n), n // 4, seed, keep_mean=True,
                                          tag=30 + c) for c in range(3)])
    return out


# ---------------------------------------- 2D periodic tanh-interface density

def interface_perturbation(n, modes, amp, seed, tag=0):
    """eta(x) = amp * eta~ / max|eta~|, eta~ = sum_{m=1..modes} a_m cos mx + b_m sin mx."""
    rng = _rng(seed, tag, n, modes)
    x = grid_1d(n)
    m = np.arange(1, modes + 1)
    et = np.cos(np.outer(x, m)) @ rng.standard_normal(modes) + \
        np.sin(np.outer(x, m)) @ rng.standard_normal(modes)
    return amp * et / np.max(np.abs(et))


def slab_density_2d(n, r, seed, width=0.05, modes=8, amp=0.1):
    """rho = 1 + (r-1)/2 [tanh((y-pi/2-eta)/w) - tanh((y-3pi/2-eta)/w)], eta = eta(x)."""
    y = grid_1d(n)[:, None]
    eta = interface_perturbation(n, modes, amp, seed, tag=4)[None, :]
    return np.ascontiguousarray(
        1.0 + 0.5 * (r - 1.0) * (np.tanh((y - np.pi / 2 - eta) / width)
                                 - np.tanh((y - 3 * np.pi / 2 - eta) / width)))


def serving_requests(count=4096, master_seed=2024, sizes=(128, 256, 512, 1024)):
    """Request descriptors for the serving stream: grid size, density ratio, seed."""
    rng = _rng(master_seed, 5)
    n = rng.choice(np.asarray(sizes), size=count)
    r = np.exp(rng.uniform(np.log(1.5), np.log(10.0), size=count))
    seeds = rng.integers(0, 2 ** 31 - 1, size=count)
    return [{"n": int(n[i]), "r": float(r[i]), "seed": int(seeds[i])} for i in range(count)]


def serving_inputs(req):
    n = req["n"]
    return {"rho": slab_density_2d(n, req["r"], req["seed"]),
            "f": band_limited((n, n), 32, req["seed"], tag=6),
            "lengths": (TWO_PI, TWO_PI)}


def slab_shape_2d(n, seed, width=0.05, modes=8, amp=0.1):
    """S(x, y) = tanh((y-pi/2-eta)/w) - tanh((y-3pi/2-eta)/w), so that the
    serving density of ratio r is 1 + (r-1)/2 S."""
    y = grid_1d(n)[:, None]
    eta = interface_perturbation(n, modes, amp, seed, tag=4)[None, :]
    return np.ascontiguousarray(np.tanh((y - np.pi / 2 - eta) / width)
                                - np.tanh((y - 3 * np.pi / 2 - eta) / width))


def serving_pool(sizes=(128, 256, 512, 1024), pool=8, seed=2024):
    """Per grid size, `pool` interface shapes and right-hand sides; request
    i uses entry (seed_i mod pool) with its own density ratio."""
    out = {}
    for n in sizes:
        out[n] = [(slab_shape_2d(n, seed + 97 * k), band_limited((n, n), 32, seed + 97 * k, tag=6))
                  for k in range(pool)]
    return out


def serving_density(shape_field, r):
    return 1.0 + 0.5 * (r - 1.0) * shape_field


def poisson_arrivals(count, qps, seed=2024):
    rng = _rng(seed, 7)
    return np.cumsum(rng.exponential(1.0 / qps, size=count))


# --------------------------------------------------- 3D multi-mode interface

def c5_density(n=512, r=10.0, width=0.02, modes=32, amp=0.1, seed=0):
    """rho = 1 + (r-1)/2 [tanh((z-pi/2-eta)/w) - tanh((z-3pi/2-eta)/w)], eta = eta(x, y)."""
    rng = _rng(seed, 8, n)
    x = grid_1d(n)
    yy, xx = np.meshgrid(x, x, indexing="ij")
    et = np.zeros((n, n))
    count = 0
    while count < modes:
        kx, ky = rng.integers(-8, 9, size=2)
        if max(abs(kx), abs(ky)) < 1:
            continue
        et += np.cos(kx * xx + ky * yy + rng.uniform(0, TWO_PI))
        count += 1
    eta = amp * et / np.max(np.abs(et))
    z = x[:, None, None]
    return np.ascontiguousarray(
        1.0 + 0.5 * (r - 1.0) * (np.tanh((z - np.pi / 2 - eta[None]) / width)
                                 - np.tanh((z - 3 * np.pi / 2 - eta[None]) / width)))


def c5_inputs(n=512, seed=0):
    return {"rho": c5_density(n, seed=seed), "f": band_limited((n, n, n), n // 4, seed, tag=9),
            "lengths": (TWO_PI,) * 3}


# ------------------------------------ 2D Fourier x Chebyshev (wall-bounded)

def cheb_gl(m):
    return np.cos(np.pi * np.arange(m + 1) / m)


def c2_inputs(nx=512, m=256, r=3.0, seed=0, lx=2.0, width=0.02):
    """rho = 1 + (r-1)/2 (1 + tanh((z - eta(x))/w)), eta 16 modes of amplitude 0.05.

    f = Re sum_{1<=|m|<=16, 0<=n<=16} c_mn exp(i pi m x) T_n(z): no x-mean
    term, so f is compatible with the Neumann walls by construction.
    Shape (m+1, nx), row 0 is z = +1.
    """
    rng = _rng(seed, 10, nx, m)
    x = lx * np.arange(nx) / nx
    z = cheb_gl(m)
    modes = np.arange(1, 17)
    et = np.cos(np.pi * np.outer(x, modes)) @ rng.standard_normal(16) + \
        np.sin(np.pi * np.outer(x, modes)) @ rng.standard_normal(16)
    eta = 0.05 * et / np.max(np.abs(et))
    rho = 1.0 + 0.5 * (r - 1.0) * (1.0 + np.tanh((z[:, None] - eta[None, :]) / width))
    th = np.arccos(np.clip(z, -1, 1))
    T = np.cos(np.outer(np.arange(17), th))           # T_n(z) = cos(n theta)
    f = np.zeros((m + 1, nx))
    for mm in list(range(-16, 0)) + list(range(1, 17)):
        c = rng.standard_normal(17) + 1j * rng.standard_normal(17)
        f += np.real(np.outer(T.T @ c, np.exp(1j * np.pi * mm * x)))
    f /= np.sqrt(np.mean(f * f))
    return {"rho": np.ascontiguousarray(rho), "f": np.ascontiguousarray(f), "lx": lx}


# ------------------------------------ batched 1D viscous systems (Sec. 3.1)

def visc1d_inputs(batch, n=257, s=1000.0, seed=0):
    """A batch of 1D viscous systems on the n Chebyshev-Gauss-Lobatto points
    (descending) of [-1, 1]: top-hat densities of eq. VDINSE.rho.hat with
    ratio s, width 0.1 and half-width x0 uniform in [0.3, 0.5] per system,
    right-hand sides standard normal with zero wall values.  Shapes (batch, n)."""
    rng = _rng(seed, 11, batch, n)
    x = cheb_gl(n - 1)
    x0 = rng.uniform(0.3, 0.5, size=(batch, 1))
    rho = 1.0 + 0.5 * (s - 1.0) * (np.tanh((x + x0) / 0.1) - np.tanh((x - x0) / 0.1))
    b = rng.standard_normal((batch, n))
    b[:, 0] = b[:, -1] = 0.0
    return {"rho": np.ascontiguousarray(rho), "b": b, "x": x}


def tophat(x, s, x0, d=0.1):
    """Top-hat density of eq. VDINSE.rho.hat centred on 0:
    1 + (s - 1)/2 [tanh((x + x0)/d) - tanh((x - x0)/d)]."""
    return 1.0 + 0.5 * (s - 1.0) * (np.tanh((x + x0) / d) - np.tanh((x - x0) / d))
