"""Seeded synthetic inputs shaped like the paper's ptychography workloads.

This module only draws random inputs: objects, probes, scan positions and
Poisson counts from given expected intensities.  It holds none of the
reconstruction method's arithmetic (no propagation, no objective, no
gradient), so the FP64 oracle and the HIP path can both consume it.

Workload shapes follow the paper's experimental setup (Results section:
2048^2 / 1024^2 objects, 4K-16K diffraction patterns, a probe of a few hundred
pixels, 128 iterations) scaled to the configurations below.  The paper's
siemens-star / coins / pillar datasets are not available; these seeded
inputs stand in for them.

Everything is generated in FP64 with numpy's PCG64 and cast by the caller.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 210607575


@dataclasses.dataclass(frozen=True)
class Config:
    """One workload: object H x W, probe n x n, a scan and a photon level."""

    name: str
    cid: int                 # config number, used to derive seeds
    obj_h: int
    obj_w: int
    n: int
    scan: str                # "raster" or "uniform"
    grid: tuple = (0, 0)     # raster rows, cols
    step: int = 0            # raster step (px)
    jitter: int = 0          # raster jitter (+-px, uniform integers)
    k_uniform: int = 0       # number of uniform random positions
    probe_kind: str = "disk"  # "gauss" (tiny case) or "disk"
    photons: float = 0.0     # sum |p|^2; 0 = unscaled (peak amplitude 1)
    noise: bool = True       # Poisson counts (True) or noise-free intensities
    iters: int = 1

    @property
    def k(self) -> int:
        if self.scan == "raster":
            return self.grid[0] * self.grid[1]
        return self.k_uniform

    def seed(self, what: str) -> int:
        off = {"object": 1, "probe": 2, "scan": 3, "poisson": 4}[what]
        return SEED_BASE + 100 * self.cid + off


CONFIGS = {
    # Tiny plain ML-CG: 128^2 object, 16^2 Gaussian probe, 8x8 raster step 8
    # +-1, noise-free intensities, 32 iterations.
    "c1": Config("c1", 1, 128, 128, 16, "raster", (8, 8), 8, 1,
                 probe_kind="gauss", photons=0.0, noise=False, iters=32),
    # Single large projection: 2048^2 object, 128^2 apodised-disk probe,
    # 64x64 raster step 24 +-2, Poisson at 1e5 photons, 100 iterations.
    "c2": Config("c2", 2, 2048, 2048, 128, "raster", (64, 64), 24, 2,
                 probe_kind="disk", photons=1e5, noise=True, iters=100),
    # Differentiable operator: 1024^2 object, 2048 uniform positions,
    # Poisson at 1e4 photons.
    "c3": Config("c3", 3, 1024, 1024, 128, "uniform", k_uniform=2048,
                 probe_kind="disk", photons=1e4, noise=True, iters=1),
    # Large one-GPU share: 8192^2 object, 256^2 probe, 128x128 raster step
    # 48 +-3, Poisson at 1e6 photons, 50 joint iterations.
    "c5": Config("c5", 5, 8192, 8192, 256, "raster", (128, 128), 48, 3,
                 probe_kind="disk", photons=1e6, noise=True, iters=50),
}


def small_config(name: str, obj: int, n: int, grid: int, step: int,
                 jitter: int, photons: float = 1e4, noise: bool = True,
                 cid: int = 90, iters: int = 8) -> Config:
    """A reduced raster workload for tests that must finish in seconds."""
    return Config(name, cid, obj, obj, n, "raster", (grid, grid), step, jitter,
                  probe_kind="disk", photons=photons, noise=noise, iters=iters)


def make_object(h: int, w: int, seed: int) -> np.ndarray:
    """complex128 transmission: amplitude U[0.9, 1.0], smooth phase in
    [-pi/4, pi/4] (white noise through a periodic Gaussian of sigma 4 px,
    applied in the Fourier domain, then an affine map of [min, max])."""
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.9, 1.0, size=(h, w))
    noise = rng.standard_normal((h, w))
    sigma = 4.0
    fy = np.fft.fftfreq(h)[:, None]
    fx = np.fft.fftfreq(w)[None, :]
    kernel = np.exp(-2.0 * (math.pi * sigma) ** 2 * (fy * fy + fx * fx))
    smooth = np.fft.ifft2(np.fft.fft2(noise) * kernel).real
    lo, hi = smooth.min(), smooth.max()
    phase = (smooth - lo) / (hi - lo) * (math.pi / 2) - math.pi / 4
    return amp * np.exp(1j * phase)


def make_probe(n: int, kind: str, photons: float, seed: int) -> np.ndarray:
    """complex128 n x n probe.

    gauss: amplitude exp(-r^2 / 2 sigma^2), sigma 4, peak 1, times a random
    quadratic phase exp(i alpha r^2), alpha = phi_e / (2 sigma)^2,
    phi_e ~ U[pi, 2 pi].
    disk: amplitude 1 inside radius R = n/4, Gaussian edge of width w = n/32
    beyond, times exp(i alpha r^2), alpha = phi_e / R^2, phi_e ~ U[2pi, 4pi].
    If photons > 0 the probe is scaled so that sum |p|^2 = photons.
    """
    rng = np.random.default_rng(seed)
    c = (n - 1) / 2.0
    yy, xx = np.meshgrid(np.arange(n) - c, np.arange(n) - c, indexing="ij")
    r2 = yy * yy + xx * xx
    if kind == "gauss":
        sigma = 4.0
        amp = np.exp(-r2 / (2 * sigma * sigma))
        phi_e = rng.uniform(math.pi, 2 * math.pi)
        alpha = phi_e / (2 * sigma) ** 2
    elif kind == "disk":
        rad = n / 4.0
        wid = n / 32.0
        r = np.sqrt(r2)
        amp = np.where(r <= rad, 1.0, np.exp(-((r - rad) ** 2) / (2 * wid * wid)))
        phi_e = rng.uniform(2 * math.pi, 4 * math.pi)
        alpha = phi_e / rad ** 2
    else:
        raise ValueError(f"unknown probe kind {kind!r}")
    p = amp * np.exp(1j * alpha * r2)
    if photons > 0:
        p = p * math.sqrt(photons / np.sum(np.abs(p) ** 2))
    return p


def make_scan(cfg: Config, seed: int) -> np.ndarray:
    """int32 [k, 2] (row, col) top-left corners, all patches inside the object.

    raster: r = o + i*step + J, c = o' + j*step + J', J ~ U{-jit..jit},
    o = floor((H - ((n_rows-1)*step + N)) / 2), row-major order.
    uniform: positions uniform on {0..H-N} x {0..W-N}.
    """
    rng = np.random.default_rng(seed)
    if cfg.scan == "raster":
        nr, nc = cfg.grid
        o_r = (cfg.obj_h - ((nr - 1) * cfg.step + cfg.n)) // 2
        o_c = (cfg.obj_w - ((nc - 1) * cfg.step + cfg.n)) // 2
        ii, jj = np.meshgrid(np.arange(nr), np.arange(nc), indexing="ij")
        jr = rng.integers(-cfg.jitter, cfg.jitter + 1, size=(nr, nc))
        jc = rng.integers(-cfg.jitter, cfg.jitter + 1, size=(nr, nc))
        rows = o_r + ii * cfg.step + jr
        cols = o_c + jj * cfg.step + jc
        pos = np.stack([rows.ravel(), cols.ravel()], axis=1)
    elif cfg.scan == "uniform":
        rows = rng.integers(0, cfg.obj_h - cfg.n + 1, size=cfg.k_uniform)
        cols = rng.integers(0, cfg.obj_w - cfg.n + 1, size=cfg.k_uniform)
        pos = np.stack([rows, cols], axis=1)
    else:
        raise ValueError(cfg.scan)
    pos = pos.astype(np.int32)
    if (pos.min() < 0 or pos[:, 0].max() > cfg.obj_h - cfg.n
            or pos[:, 1].max() > cfg.obj_w - cfg.n):
        raise ValueError("scan leaves the object")
    return pos


def poisson_counts(intensity: np.ndarray, seed: int, chunk: int = 256) -> np.ndarray:
    """float32 Poisson draws with the given expected intensities [k, n, n].

    Chunks of `chunk` patterns each use a child of SeedSequence(seed), so the
    result does not depend on how the caller batches its intensities."""
    k = intensity.shape[0]
    out = np.empty(intensity.shape, dtype=np.float32)
    nchunks = (k + chunk - 1) // chunk
    children = np.random.SeedSequence(seed).spawn(nchunks)
    for ci in range(nchunks):
        lo, hi = ci * chunk, min(k, (ci + 1) * chunk)
        rng = np.random.default_rng(children[ci])
        out[lo:hi] = rng.poisson(np.maximum(intensity[lo:hi], 0.0)).astype(np.float32)
    return out


@dataclasses.dataclass
class Inputs:
    cfg: Config
    obj_true: np.ndarray     # complex128 [H, W]
    probe: np.ndarray        # complex128 [n, n]
    pos: np.ndarray          # int32 [k, 2]


def make_inputs(cfg: Config) -> Inputs:
    """Object (ground truth), probe and scan of a configuration.  The
    measured intensities need the forward model, which the caller supplies
    (see `make_data`)."""
    return Inputs(cfg,
                  make_object(cfg.obj_h, cfg.obj_w, cfg.seed("object")),
                  make_probe(cfg.n, cfg.probe_kind, cfg.photons, cfg.seed("probe")),
                  make_scan(cfg, cfg.seed("scan")))


def make_data(cfg: Config, intensity: np.ndarray) -> np.ndarray:
    """Measured intensities from expected intensities |G psi_true|^2 computed
    by the caller's forward model: noise-free (float64) or Poisson (float32)."""
    if cfg.noise:
        return poisson_counts(intensity, cfg.seed("poisson"))
    return np.asarray(intensity, dtype=np.float64)


def initial_object(cfg: Config) -> np.ndarray:
    """The CG starting guess: all ones."""
    return np.ones((cfg.obj_h, cfg.obj_w), dtype=np.complex128)
