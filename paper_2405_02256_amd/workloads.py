"""Seeded synthetic inputs for the five workloads and for tiny test cases.

This module only draws random numbers and shapes arrays.  It holds none of
the transform arithmetic (no cells, no Euler characteristics, no projections),
so both the CPU oracle and the GPU path can consume its output without sharing
any of the method's code.

Every generator uses numpy's PCG64 ``default_rng(seed)``; ``digest()`` gives a
SHA-256 of any array so that a run can record exactly what it consumed.

Workloads (sizes follow the method's use on images and volumes):

* ``small_binary``    64x64 majority-filtered Bernoulli(0.5) image, 64 ECT
                      directions x 64 thresholds, 256 Euler-Fourier vectors.
* ``grf_512``         512x512 Gaussian random field (sigma 8 px) thresholded
                      at its median; 360 ECT directions x 256 thresholds and
                      4096 hybrid vectors with |xi| ~ U[0.01, 1].
* ``volume_128``      128^3 smoothed noise quantised to 8 levels; 2048
                      Fibonacci-sphere directions x 256 thresholds and 16384
                      hybrid vectors with |xi| ~ U[0.01, 4], corner origin.
* ``batch_4096``      4096 ragged binary fields with sides in {28,64,128,256};
                      128 directions x 128 thresholds and 512 Laplace vectors
                      per image.
* ``diff_256``        256 binary fields 128x128 with 1024 shared learnable
                      vectors kept away from the coordinate axes.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np
from scipy import ndimage

PRIMAL = 0  # pixels are top-dimensional cells, lower cells take the min of their cofaces
DUAL = 1    # pixels are vertices, higher cells take the min of their vertices


def digest(a: np.ndarray) -> str:
    a = np.ascontiguousarray(a)
    h = hashlib.sha256()
    h.update(str(a.dtype).encode())
    h.update(str(a.shape).encode())
    h.update(a.tobytes())
    return h.hexdigest()


# --------------------------------------------------------------------------
# image generators (arrays are indexed [axis_{n-1}, ..., axis_0]: axis 0 is the
# fastest-varying memory axis, i.e. numpy's last index)
# --------------------------------------------------------------------------

def bernoulli_majority(rng: np.random.Generator, side: int) -> np.ndarray:
    """Bernoulli(0.5) pixels followed by one 3x3 majority filter (zero padding)."""
    px = (rng.random((side, side)) < 0.5).astype(np.int32)
    box = ndimage.convolve(px, np.ones((3, 3), np.int32), mode="constant", cval=0)
    return (box >= 5).astype(np.uint8)


def gaussian_field(rng: np.random.Generator, shape, sigma: float) -> np.ndarray:
    """Standard normal noise smoothed by a separable Gaussian (radius ceil(4 sigma), reflect)."""
    noise = rng.standard_normal(shape)
    return ndimage.gaussian_filter(noise, sigma=sigma, mode="reflect", truncate=4.0)


def binary_field(rng: np.random.Generator, shape, sigma: float) -> np.ndarray:
    """Gaussian random field thresholded at its median ("value > median")."""
    f = gaussian_field(rng, shape, sigma)
    return (f > np.median(f)).astype(np.uint8)


def quantised_field(rng: np.random.Generator, shape, sigma: float, levels: int = 8) -> np.ndarray:
    """Smoothed noise of any shape; each element holds the number of level cuts below it (0..levels-1)."""
    f = gaussian_field(rng, shape, sigma)
    cuts = np.quantile(f, np.arange(1, levels) / levels)
    return np.searchsorted(cuts, f, side="right").astype(np.uint8)


def quantised_volume(rng: np.random.Generator, side: int, sigma: float, levels: int = 8) -> np.ndarray:
    """Smoothed noise volume; each voxel holds the number of level cuts below it (0..levels-1)."""
    return quantised_field(rng, (side, side, side), sigma, levels)


# --------------------------------------------------------------------------
# query generators
# --------------------------------------------------------------------------

def circle_dirs(count: int) -> np.ndarray:
    k = np.arange(count, dtype=np.float64)
    th = 2.0 * np.pi * k / count
    return np.stack([np.cos(th), np.sin(th)], axis=1)


def fibonacci_dirs(count: int) -> np.ndarray:
    k = np.arange(count, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / count
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    ph = k * np.pi * (3.0 - np.sqrt(5.0))
    return np.stack([r * np.cos(ph), r * np.sin(ph), z], axis=1)


def even_thresholds(radius: float, count: int) -> np.ndarray:
    j = np.arange(count, dtype=np.float64)
    return -radius + j * (2.0 * radius / (count - 1))


def polar_vectors(rng: np.random.Generator, count: int, rmin: float, rmax: float,
                  axis_gap: float = 0.0) -> np.ndarray:
    """2D vectors with angle ~ U[0, 2pi) and norm ~ U[rmin, rmax].

    With ``axis_gap`` > 0, angles closer than that many radians to a coordinate
    axis are redrawn (the transforms have kinks where a coordinate is zero).
    """
    th = rng.uniform(0.0, 2.0 * np.pi, count)
    if axis_gap > 0.0:
        while True:
            d = np.abs(((th + np.pi / 4) % (np.pi / 2)) - np.pi / 4)
            bad = d < axis_gap
            if not bad.any():
                break
            th[bad] = rng.uniform(0.0, 2.0 * np.pi, int(bad.sum()))
    r = rng.uniform(rmin, rmax, count)
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def sphere_vectors(rng: np.random.Generator, count: int, rmin: float, rmax: float, dim: int = 3) -> np.ndarray:
    """Vectors with a uniform direction on the unit sphere of R^dim and norm ~ U[rmin, rmax]."""
    g = rng.standard_normal((count, dim))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    r = rng.uniform(rmin, rmax, count)
    return g * r[:, None]


# --------------------------------------------------------------------------
# workload records
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    ndim: int
    images: list                      # list of numpy arrays, numpy order (axis 0 last)
    construction: int = PRIMAL
    origin: np.ndarray | None = None  # [num_images][ndim] in embedding-axis order, or None = centred
    spacing: np.ndarray | None = None
    ect_dirs: np.ndarray | None = None      # [D][ndim] shared, or None
    ect_thresholds: np.ndarray | None = None  # [M] shared or [num_images][M]
    hybrid_xi: np.ndarray | None = None     # [Q][ndim] shared or [num_images*Q][ndim] ragged
    hybrid_xi_per_image: bool = False
    hybrid_kernels: tuple = ()
    hybrid_s: float = 1.0
    meta: dict = field(default_factory=dict)

    def dims(self) -> np.ndarray:
        """[num_images][ndim] pixel counts in embedding-axis order (axis 0 first)."""
        return np.array([list(reversed(im.shape)) for im in self.images], dtype=np.int32)

    def pixels_concat(self):
        """Concatenated uint8 pixels (each image C-contiguous) and element offsets."""
        flat = [np.ascontiguousarray(im).reshape(-1) for im in self.images]
        offs = np.zeros(len(flat), dtype=np.int64)
        if len(flat) > 1:
            offs[1:] = np.cumsum([f.size for f in flat[:-1]])
        return np.concatenate(flat), offs

    def digests(self) -> dict:
        px, _ = self.pixels_concat()
        d = {"pixels": digest(px)}
        if self.ect_dirs is not None:
            d["ect_dirs"] = digest(self.ect_dirs)
        if self.hybrid_xi is not None:
            d["hybrid_xi"] = digest(self.hybrid_xi)
        return d


def small_binary(seed: int = 1) -> Workload:
    rng = np.random.default_rng(seed)
    img = bernoulli_majority(rng, 64)
    R = 32.0 * math.sqrt(2.0)
    a = np.arange(16, dtype=np.float64)
    om = 0.05 * 40.0 ** (a / 15.0)
    th = 2.0 * np.pi * np.arange(16, dtype=np.float64) / 16.0
    W, T = np.meshgrid(om, th, indexing="ij")
    xi = np.stack([(W * np.cos(T)).ravel(), (W * np.sin(T)).ravel()], axis=1)
    return Workload("small_binary_64", 2, [img], ect_dirs=circle_dirs(64),
                    ect_thresholds=even_thresholds(R, 64), hybrid_xi=xi,
                    hybrid_kernels=("fourier",), meta={"R": R, "seed": seed})


def grf_512(seed: int = 2, n_xi: int = 4096) -> Workload:
    rng = np.random.default_rng(seed)
    img = binary_field(rng, (512, 512), 8.0)
    R = 256.0 * math.sqrt(2.0)
    xi = polar_vectors(rng, n_xi, 0.01, 1.0)
    return Workload("grf_512", 2, [img], ect_dirs=circle_dirs(360),
                    ect_thresholds=even_thresholds(R, 256), hybrid_xi=xi,
                    hybrid_kernels=("fourier", "laplace", "bessel"), meta={"R": R, "seed": seed})


def volume_128(seed: int = 3, side: int = 128, n_dirs: int = 2048, n_xi: int = 16384,
               sigma: float = 4.0) -> Workload:
    rng = np.random.default_rng(seed)
    vol = quantised_volume(rng, side, sigma)
    R = side * math.sqrt(3.0)
    xi = sphere_vectors(rng, n_xi, 0.01, 4.0)
    return Workload(f"volume_{side}", 3, [vol], origin=np.zeros((1, 3)),
                    ect_dirs=fibonacci_dirs(n_dirs), ect_thresholds=even_thresholds(R, 256),
                    hybrid_xi=xi, hybrid_kernels=("fourier", "laplace"),
                    meta={"R": R, "seed": seed, "sigma": sigma})


def hypervolume_24(seed: int = 6, side: int = 24, n_dirs: int = 512, n_xi: int = 4096,
                   sigma: float = 2.0) -> Workload:
    """A four-axis field (n-dimensional arrays): side^4 smoothed noise quantised into 8 levels,
    primal construction, centred; ECT at 512 uniform directions of S^3 x 256 thresholds; the
    three hybrid kernels at 4096 xi with |xi| ~ U[0.01, 1]."""
    rng = np.random.default_rng(seed)
    vol = quantised_field(rng, (side,) * 4, sigma)
    R = float(side)   # half the diagonal of the centred box [-side/2, side/2]^4
    dirs = sphere_vectors(rng, n_dirs, 1.0, 1.0, dim=4)
    xi = sphere_vectors(rng, n_xi, 0.01, 1.0, dim=4)
    return Workload(f"hypervolume_{side}", 4, [vol], ect_dirs=dirs, ect_thresholds=even_thresholds(R, 256),
                    hybrid_xi=xi, hybrid_kernels=("fourier", "laplace", "bessel"),
                    meta={"R": R, "seed": seed, "sigma": sigma})


def batch_4096(seed: int = 4, count: int = 4096, sides=(28, 64, 128, 256),
               n_dirs: int = 128, n_thr: int = 128, n_xi: int = 512) -> Workload:
    rng = np.random.default_rng(seed)
    side = rng.choice(np.asarray(sides), size=count)
    sig = rng.uniform(2.0, 8.0, size=count)
    imgs = [binary_field(rng, (int(s), int(s)), float(g)) for s, g in zip(side, sig)]
    thr = np.stack([even_thresholds(float(s) / math.sqrt(2.0), n_thr) for s in side])
    xi = np.concatenate([polar_vectors(rng, n_xi, 0.01, 1.0) for _ in range(count)])
    return Workload(f"batch_{count}", 2, imgs, ect_dirs=circle_dirs(n_dirs), ect_thresholds=thr,
                    hybrid_xi=xi, hybrid_xi_per_image=True, hybrid_kernels=("laplace",),
                    meta={"seed": seed, "sides": side.tolist(), "sigmas": sig.tolist()})


def diff_256(seed: int = 5, count: int = 256, side: int = 128, n_xi: int = 1024) -> Workload:
    rng = np.random.default_rng(seed)
    sig = rng.uniform(2.0, 8.0, size=count)
    imgs = [binary_field(rng, (side, side), float(g)) for g in sig]
    xi = polar_vectors(rng, n_xi, 0.01, 0.5, axis_gap=0.02)
    w = rng.standard_normal((count, n_xi, 2))
    return Workload(f"diff_{count}", 2, imgs, hybrid_xi=xi,
                    hybrid_kernels=("fourier", "laplace"), meta={"seed": seed, "loss_weights": w})


WORKLOADS = {
    "small_binary": small_binary,
    "grf_512": grf_512,
    "volume_128": volume_128,
    "batch_4096": batch_4096,
    "diff_256": diff_256,
}


# --------------------------------------------------------------------------
# tiny inputs for exhaustive and property tests
# --------------------------------------------------------------------------

def all_binary_images(shape) -> np.ndarray:
    """Every binary image of the given numpy shape, stacked: [2^size, *shape]."""
    size = int(np.prod(shape))
    codes = np.arange(1 << size, dtype=np.int64)
    bits = (codes[:, None] >> np.arange(size)[None, :]) & 1
    return bits.reshape((1 << size,) + tuple(shape)).astype(np.uint8)


def random_image(rng: np.random.Generator, shape, levels: int) -> np.ndarray:
    return rng.integers(0, levels, size=shape).astype(np.uint8)


# The 4x4 binary image of the method's running example (dual construction);
# row j is embedding axis 1, column i is embedding axis 0.
RUNNING_EXAMPLE = np.array([[1, 0, 0, 0],
                            [0, 1, 1, 0],
                            [1, 1, 1, 1],
                            [1, 1, 0, 0]], dtype=np.uint8)
