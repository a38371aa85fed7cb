"""Seeded synthetic workloads: random fields, sampling masks, ragged batches.

This module only makes inputs.  It holds none of the gap-filling method's
arithmetic (no angle map, no energy, no Monte Carlo); the HIP path, the oracle
and the benchmark all draw their inputs from here so that they see the same
numbers.

Fields follow the paper's experiments (Section 4): Gaussian random fields with
the Whittle-Matern covariance (equation "mate"), simulated by a spectral
method.  The spectral method used here is circulant embedding: the covariance
is sampled on a periodic grid twice the image size in each direction, its
discrete Fourier transform gives the eigenvalues (negative ones, which only
appear for correlation lengths comparable to the image, are set to zero), and
the field is the real part of the transform of scaled complex white noise.
The image is the corner of that periodic field.

Sampling masks are ``uint8`` arrays with 1 at sampled (kept) sites and 0 at
gaps.  Arrays are row-major with x fastest: ``a[y, x]``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.fft
import scipy.special


def matern_cov(h: np.ndarray, nu: float, kappa: float, sigma: float) -> np.ndarray:
    """Whittle-Matern covariance at distances ``h`` (equation "mate")."""
    h = np.asarray(h, dtype=np.float64)
    out = np.empty_like(h)
    zero = h == 0.0
    x = kappa * h[~zero]
    out[~zero] = (sigma * sigma * 2.0 ** (1.0 - nu) / scipy.special.gamma(nu)
                  * x ** nu * scipy.special.kv(nu, x))
    out[zero] = sigma * sigma
    return out


def matern_field(nx: int, ny: int, nu: float, kappa: float, mean: float,
                 std: float, seed: int) -> np.ndarray:
    """Gaussian field of shape (ny, nx) with Whittle-Matern covariance."""
    n1, n2 = 2 * ny, 2 * nx
    # Distances on the torus only depend on the folded offsets, so evaluate
    # the covariance on one quadrant and index it.
    d1 = np.minimum(np.arange(n1), n1 - np.arange(n1))
    d2 = np.minimum(np.arange(n2), n2 - np.arange(n2))
    q1 = np.arange(ny + 1, dtype=np.float64)
    q2 = np.arange(nx + 1, dtype=np.float64)
    quad = matern_cov(np.hypot(q1[:, None], q2[None, :]), nu, kappa, std)
    base = quad[d1[:, None], d2[None, :]]
    lam = scipy.fft.fft2(base, workers=-1).real
    del base
    np.maximum(lam, 0.0, out=lam)
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((n1, n2)) + 1j * rng.standard_normal((n1, n2))
    noise *= np.sqrt(lam / (n1 * n2))
    del lam
    f = scipy.fft.fft2(noise, workers=-1, overwrite_x=True)
    return np.ascontiguousarray(f.real[:ny, :nx]) + mean


def lognormal_field(nx: int, ny: int, nu: float, kappa: float, log_std: float,
                    seed: int) -> np.ndarray:
    """exp(G) with G a zero-mean Whittle-Matern Gaussian field."""
    return np.exp(matern_field(nx, ny, nu, kappa, 0.0, log_std, seed))


def random_mask(nx: int, ny: int, p_removed: float, seed: int) -> np.ndarray:
    """Remove exactly round(p * nx * ny) sites, chosen uniformly at random."""
    n = nx * ny
    n_gap = int(round(p_removed * n))
    rng = np.random.default_rng(seed)
    mask = np.ones(n, dtype=np.uint8)
    mask[rng.permutation(n)[:n_gap]] = 0
    return mask.reshape(ny, nx)


def cloud_mask(nx: int, ny: int, p_removed: float, seed: int,
               nu: float = 1.5, kappa: float = 0.02) -> np.ndarray:
    """Contiguous gaps: the sites where an independent Matern field is lowest.

    Exactly round(p * nx * ny) sites are removed (the field's lower quantile).
    """
    w = matern_field(nx, ny, nu, kappa, 0.0, 1.0, seed).ravel()
    n_gap = int(round(p_removed * w.size))
    mask = np.ones(w.size, dtype=np.uint8)
    if n_gap > 0:
        idx = np.argpartition(w, n_gap - 1)[:n_gap]
        mask[idx] = 0
    return mask.reshape(ny, nx)


@dataclass
class Image:
    """One synthetic gap-filling problem."""
    z: np.ndarray          # (ny, nx) float64 true field
    mask: np.ndarray       # (ny, nx) uint8, 1 = sampled
    name: str

    @property
    def nx(self) -> int:
        return self.z.shape[1]

    @property
    def ny(self) -> int:
        return self.z.shape[0]


# Seeds: field 1000+c, mask 2000+c, Monte Carlo 3000+c for workload c.
def seeds(c: int) -> tuple[int, int, int]:
    return 1000 + c, 2000 + c, 3000 + c


def workload_l64() -> Image:
    """64x64 Gaussian WM nu=0.5 kappa=0.2, mean 50, std 10, 33% removed."""
    fs, ms, _ = seeds(0)
    z = matern_field(64, 64, 0.5, 0.2, 50.0, 10.0, fs)
    return Image(z, random_mask(64, 64, 0.33, ms), "wm_l64_p33")


def workload_l1024() -> Image:
    """1024x1024 Gaussian WM nu=2.5 kappa=0.05, mean 50, std 10, 50% removed."""
    fs, ms, _ = seeds(1)
    z = matern_field(1024, 1024, 2.5, 0.05, 50.0, 10.0, fs)
    return Image(z, random_mask(1024, 1024, 0.5, ms), "wm_l1024_p50")


def workload_l4096(mask_kind: str = "random", n: int = 4096) -> Image:
    """Lognormal exp(G), G WM nu=1.5 kappa=0.02 std 0.5; 66% random or 40% cloud."""
    fs, ms, _ = seeds(2)
    z = lognormal_field(n, n, 1.5, 0.02, 0.5, fs)
    if mask_kind == "random":
        m = random_mask(n, n, 0.66, ms)
    elif mask_kind == "cloud":
        m = cloud_mask(n, n, 0.40, ms)
    else:
        raise ValueError(mask_kind)
    return Image(z, m, f"lognormal_l{n}_{mask_kind}")


def workload_table2(n: int, p_removed: float, rep: int) -> Image:
    """Section 4 set-up: WM nu=0.5 kappa=0.2, N(50, 10), random removal."""
    z = matern_field(n, n, 0.5, 0.2, 50.0, 10.0, 5000 + rep)
    return Image(z, random_mask(n, n, p_removed, 6000 + rep), f"t2_l{n}_{rep}")


def _ragged_image(spec: tuple) -> Image:
    nx, ny, nu, kappa, p, seed, i = spec
    z = matern_field(nx, ny, nu, kappa, 50.0, 10.0, seed * 1000 + i)
    m = random_mask(nx, ny, p, seed * 1000 + 500 + i)
    return Image(z, m, f"ragged_{i}_{nx}x{ny}")


def ragged_batch(n_images: int = 256, lo: int = 128, hi: int = 2048,
                 seed: int = 1003, workers: int = 1) -> list[Image]:
    """Images of uneven size: sides log-uniform integers in [lo, hi].

    nu from {0.5, 1.5, 2.5}, kappa log-uniform in [0.01, 0.3], mean 50,
    std 10, removal fraction uniform in [0.2, 0.8], random masks.  With
    workers > 1 the images are made in that many fresh processes (the
    result does not depend on it).
    """
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n_images):
        nx = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        ny = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        nu = float(rng.choice([0.5, 1.5, 2.5]))
        kappa = float(math.exp(rng.uniform(math.log(0.01), math.log(0.3))))
        p = float(rng.uniform(0.2, 0.8))
        specs.append((nx, ny, nu, kappa, p, seed, i))
    if workers <= 1:
        return [_ragged_image(sp) for sp in specs]
    import concurrent.futures
    import multiprocessing
    # largest first, so that the pool's tail is short
    order = sorted(range(n_images), key=lambda k: -specs[k][0] * specs[k][1])
    with concurrent.futures.ProcessPoolExecutor(max_workers=workers,
                                                mp_context=multiprocessing.get_context("spawn")) as ex:
        made = list(ex.map(_ragged_image, [specs[k] for k in order]))
    out = [None] * n_images
    for k, im in zip(order, made):
        out[k] = im
    return out


def validation_measures(z_true: np.ndarray, z_hat: np.ndarray,
                        mask: np.ndarray) -> dict:
    """MAAE, MARE [%], MAARE [%], MRASE over gap sites with error z - z_hat."""
    g = mask == 0
    eps = z_true[g] - z_hat[g]
    zt = z_true[g]
    return {
        "MAAE": float(np.mean(np.abs(eps))),
        "MARE": float(np.mean(eps / zt) * 100.0),
        "MAARE": float(np.mean(np.abs(eps / zt)) * 100.0),
        "MRASE": float(np.sqrt(np.mean(eps * eps))),
    }
