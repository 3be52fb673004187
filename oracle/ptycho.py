"""FP64 CPU oracle for maximum-likelihood CG ptychography.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow reference the HIP
path is checked against.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the product path never does.
It shares no code with the HIP path (no kernels, tables, helpers or pre/post
processing); the only common module is the seeded input generator, which
holds none of the method's arithmetic.

Every function below follows one passage of the paper (arXiv 2106.07575,
section "Background", subsections "Forward problem of ptychography" and
"Inverse problem for ptychography", Eqs. fwd_model, ML, gradient, update2
(gradient descent), update, DaiYuan, linesearch; the CG coefficient eq. cg_ch1_1 of section "Challenges
of CG solver parallelization"; and Algorithm 1, "Complete workflow of
PtyGer").  Precision is complex128 / float64 throughout.

Readings where the paper is silent or ambiguous (each is listed with its
reason in the design notes):
  * F is the unitary 2-D DFT (1/N per N x N transform), DC at [0, 0], no
    shift; F^H is then both the adjoint and the inverse, as the paper states.
  * d holds measured intensities, |G psi|^2 = d.
  * log|g| and d/conj(g) are guarded by x = |g|^2 >= eps (eps = 1e-32); below
    the guard the residual is g and the log uses eps.
  * The line search compares the deviance Phi = F - C (C = sum over d > 0 of
    d - d log d), which differs from Eq. ML by a constant; both are reported.
  * <a, b> = sum conj(a) b is complex; the Dai-Yuan denominator uses its real
    part.  A non-positive or non-finite denominator restarts (beta = 0).
  * The line search shrinks gamma before the first trial (gamma0 * tau first,
    as in Algorithm 1) and stops when the Eq. linesearch condition holds;
    after `lmax` failed trials gamma = 0 and the next direction restarts.
  * Scan positions are integer (row, col) top-left corners inside the object.
  * Joint object+probe mode (not in the paper) runs the same CG on the pair
    (psi, p) with inner products summed over both blocks.
  * The least-squares estimator, which the paper says its techniques also
    apply to but gives no formula for, is taken as F = sum (|g| - sqrt d)^2
    with the Wirtinger gradient convention of Eq. gradient.

Parity status: every function here is pinned by the not-gpu tests (brute
force DFT, closed forms, adjoint identity, zero gradient at the truth, finite
differences, hand-computed Dai-Yuan coefficients, line-search semantics).
The whole CG trajectory has no printed value to pin it: beyond its
invariants (monotone objective, descent directions, convergence toward the
truth) it is "parity unpinned".
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft

EPS = 1e-32          # guard on |g|^2 (reading of Eqs. ML / gradient at g = 0)
CHUNK = 256          # patterns per FFT batch (memory only; no reordering)
_WORKERS = os.cpu_count() or 1


# ---------------------------------------------------------------- transforms
def fft2u(x: np.ndarray) -> np.ndarray:
    """Unitary forward 2-D DFT over the last two axes:
    X[a, b] = (1/N) sum_{u,v} x[u, v] exp(-2 pi i (a u + b v) / N)."""
    return scipy.fft.fft2(np.asarray(x, dtype=np.complex128), norm="ortho",
                          workers=_WORKERS)


def ifft2u(x: np.ndarray) -> np.ndarray:
    """Unitary inverse 2-D DFT (= adjoint of fft2u), the paper's F^H."""
    return scipy.fft.ifft2(np.asarray(x, dtype=np.complex128), norm="ortho",
                           workers=_WORKERS)


def dft2_bruteforce(x: np.ndarray, inverse: bool = False) -> np.ndarray:
    """The unitary 2-D DFT written out as its quadruple sum (small n only).

    Used to pin fft2u / ifft2u: X[a,b] = (1/n) sum_u sum_v x[u,v] w^(a u + b v)
    with w = exp(-+ 2 pi i / n)."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[-1]
    assert x.shape[-2] == n and n <= 32
    sign = 1.0 if inverse else -1.0
    out = np.zeros_like(x)
    for a in range(n):
        for b in range(n):
            acc = np.zeros(x.shape[:-2], dtype=np.complex128)
            for u in range(n):
                for v in range(n):
                    acc = acc + x[..., u, v] * np.exp(sign * 2j * math.pi * (a * u + b * v) / n)
            out[..., a, b] = acc / n
    return out


# ------------------------------------------------------- Q and Q^H (Eq. 1, 3)
def gather(obj: np.ndarray, pos: np.ndarray, n: int) -> np.ndarray:
    """Patches psi[r_k : r_k + n, c_k : c_k + n] for every scan position."""
    pos = np.asarray(pos)
    out = np.empty((pos.shape[0], n, n), dtype=obj.dtype)
    for k, (r, c) in enumerate(pos):
        out[k] = obj[r:r + n, c:c + n]
    return out


def scatter_add(patches: np.ndarray, pos: np.ndarray, shape) -> np.ndarray:
    """Sum of patches placed at their scan positions (k in increasing order)."""
    n = patches.shape[-1]
    out = np.zeros(shape, dtype=patches.dtype)
    for k, (r, c) in enumerate(np.asarray(pos)):
        out[r:r + n, c:c + n] += patches[k]
    return out


def illumination(probe: np.ndarray, pos: np.ndarray, shape) -> np.ndarray:
    """sum_k |p(. - s_k)|^2 on the object grid (diagonal of G^H G)."""
    pk = np.broadcast_to(np.abs(probe) ** 2, (len(pos),) + probe.shape)
    return scatter_add(np.ascontiguousarray(pk), pos, shape)


# ------------------------------------------------------------------ G, G^H
def forward(obj: np.ndarray, probe: np.ndarray, pos: np.ndarray) -> np.ndarray:
    """Eq. fwd_model: g_k = F (p * psi[s_k]) for every position, [k, n, n]."""
    n = probe.shape[0]
    out = np.empty((len(pos), n, n), dtype=np.complex128)
    for lo in range(0, len(pos), CHUNK):
        sl = slice(lo, lo + CHUNK)
        out[sl] = fft2u(probe[None] * gather(obj, pos[sl], n))
    return out


def adjoint(far: np.ndarray, probe: np.ndarray, pos: np.ndarray, shape,
            obj: np.ndarray | None = None):
    """G^H = Q^H F^H (text after Eq. gradient).

    Returns (obj_out, probe_out): obj_out = sum_k place_k(conj(p) * F^H far_k);
    probe_out = sum_k conj(psi[s_k]) * F^H far_k when `obj` is given, else None.
    """
    n = probe.shape[0]
    obj_out = np.zeros(shape, dtype=np.complex128)
    probe_out = None if obj is None else np.zeros((n, n), dtype=np.complex128)
    for lo in range(0, len(pos), CHUNK):
        sl = slice(lo, lo + CHUNK)
        u = ifft2u(far[sl])
        obj_out += scatter_add(np.conj(probe)[None] * u, pos[sl], shape)
        if obj is not None:
            probe_out += np.sum(np.conj(gather(obj, pos[sl], n)) * u, axis=0)
    return obj_out, probe_out


# ------------------------------------------------------- objective (Eq. 2)
def objective_terms(x: np.ndarray, d: np.ndarray, eps: float = EPS, estimator: str = "ml"):
    """Per-pixel terms of the objective for intensities x = |g|^2.

    estimator "ml" (Eq. ML):
      paper: x - d log max(x, eps)            (2 d log|g| = d log|g|^2)
      dev:   x - d - d log(max(x, eps) / d)   for d > 0;  x for d = 0
      Both drop d log(.) where d = 0.  dev = paper - (d - d log d).
    estimator "ls" (least squares on amplitudes; the paper names the LS
    estimate without a formula, the usual one is taken):
      paper = dev = (sqrt(x) - sqrt(d))^2 for d > 0; x for d <= 0."""
    x = np.asarray(x, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    if estimator == "ls":
        t = np.where(d > 0, (np.sqrt(x) - np.sqrt(np.maximum(d, 0.0))) ** 2, x)
        return t, t
    if estimator != "ml":
        raise ValueError(f"unknown estimator {estimator!r}")
    xg = np.maximum(x, eps)
    pos = d > 0
    dsafe = np.where(pos, d, 1.0)
    paper = x - np.where(pos, d * np.log(xg), 0.0)
    dev = np.where(pos, x - d - d * np.log(xg / dsafe), x)
    return paper, dev


def residual(g: np.ndarray, d: np.ndarray, eps: float = EPS, estimator: str = "ml") -> np.ndarray:
    """Inner term of Eq. gradient: g - d / conj(g) = g (1 - d / |g|^2),
    and g where |g|^2 < eps.  Least squares: the Wirtinger derivative of
    (|g| - sqrt d)^2 with respect to conj(g), g (1 - sqrt(d) / |g|) (g where
    |g|^2 < eps or d <= 0)."""
    x = np.abs(g) ** 2
    if estimator == "ls":
        sd = np.sqrt(np.maximum(np.asarray(d, dtype=np.float64), 0.0))
        w = np.where(x >= eps, sd / np.sqrt(np.maximum(x, eps)), 0.0)
        return g * (1.0 - w)
    w = np.where(x >= eps, np.asarray(d, dtype=np.float64) / np.maximum(x, eps), 0.0)
    return g * (1.0 - w)


def minfunc(obj, probe, pos, d, eps: float = EPS, estimator: str = "ml"):
    """MINFUNC of Algorithm 1: (Phi deviance, F of Eq. ML) at psi."""
    n = probe.shape[0]
    phi = 0.0
    f = 0.0
    for lo in range(0, len(pos), CHUNK):
        sl = slice(lo, lo + CHUNK)
        g = fft2u(probe[None] * gather(obj, pos[sl], n))
        paper, dev = objective_terms(np.abs(g) ** 2, d[sl], eps, estimator)
        phi += float(np.sum(dev))
        f += float(np.sum(paper))
    return phi, f


def grad(obj, probe, pos, d, eps: float = EPS, want_probe: bool = False, estimator: str = "ml"):
    """GRAD stage (Eq. gradient): FORWARD then GRAD_COMP.

    grad_obj = G^H (g - d / conj(g)) is the Wirtinger derivative dF/d conj(psi)
    (no factor 2), so d/dh F(psi + h v) = 2 Re <grad_obj, v>.
    grad_probe = sum_k conj(psi[s_k]) * F^H r_k (joint mode).
    Returns dict(phi, f, grad_obj, grad_probe)."""
    n = probe.shape[0]
    gobj = np.zeros(obj.shape, dtype=np.complex128)
    gprb = np.zeros((n, n), dtype=np.complex128) if want_probe else None
    phi = 0.0
    f = 0.0
    for lo in range(0, len(pos), CHUNK):
        sl = slice(lo, lo + CHUNK)
        patch = gather(obj, pos[sl], n)
        g = fft2u(probe[None] * patch)
        paper, dev = objective_terms(np.abs(g) ** 2, d[sl], eps, estimator)
        phi += float(np.sum(dev))
        f += float(np.sum(paper))
        u = ifft2u(residual(g, d[sl], eps, estimator))
        gobj += scatter_add(np.conj(probe)[None] * u, pos[sl], obj.shape)
        if want_probe:
            gprb += np.sum(np.conj(patch) * u, axis=0)
    return {"phi": phi, "f": f, "grad_obj": gobj, "grad_probe": gprb}


# --------------------------------------------------------- CG (Eqs. 5-7, Alg. 1)
def inner(a: np.ndarray, b: np.ndarray) -> complex:
    """<a, b> = sum_i conj(a_i) b_i (text after Eq. DaiYuan)."""
    return complex(np.vdot(a, b))


def dai_yuan_beta(g_new, g_old, eta_old):
    """Coefficient of Eq. DaiYuan / Eq. cg_ch1_1:
    beta = ||g_new||^2 / Re <eta_old, g_new - g_old>.

    g_new etc. are tuples of blocks (object, or object and probe); the inner
    products sum over the blocks.  Returns (beta, restarted): a denominator
    that is not positive and finite gives beta = 0 (steepest descent)."""
    num = sum(inner(a, a).real for a in g_new)
    den = sum(inner(e, gn - go).real for e, gn, go in zip(eta_old, g_new, g_old))
    if not (math.isfinite(den) and den > 0.0 and math.isfinite(num)):
        return 0.0, True
    return num / den, False


def line_search(phi_of_gamma, phi_m: float, gamma0: float = 1.0,
                tau: float = 0.5, t: float = 0.0, lmax: int = 40, values=None):
    """Backtracking of Eq. linesearch in Algorithm 1's order: gamma <- tau
    gamma, evaluate, until F(psi + gamma eta) <= F(psi) + gamma t.

    Returns (gamma, trials, accepted); if `lmax` trials fail, gamma = 0.
    values (optional list): receives every trial's objective, in order."""
    gamma = gamma0
    for j in range(1, lmax + 1):
        gamma = gamma * tau
        phi_t = phi_of_gamma(gamma)
        if values is not None:
            values.append(phi_t)
        if phi_t <= phi_m + gamma * t:
            return gamma, j, True
    return 0.0, lmax, False


def cg_solve(obj0, probe0, pos, d, iters: int, gamma0: float = 1.0,
             tau: float = 0.5, t: float = 0.0, lmax: int = 40,
             eps: float = EPS, update_probe: bool = False,
             target_phi: float | None = None, estimator: str = "ml",
             callback=None):
    """ML-CG reconstruction of Algorithm 1 on one device.

    Each iteration: GRAD (Eq. gradient) -> DIR (Eq. DaiYuan, eta_0 = -grad_0)
    -> LS (Eq. linesearch) -> Update (Eq. update).  Object only (the paper)
    or joint object+probe.  Returns (obj, probe, trace) with one trace row
    per iteration: phi, f (at psi_m), gamma, halvings, beta, step_norm
    (||psi_{m+1} - psi_m||, the paper's convergence 2-norm), restarted, and
    trial_phis (the objective of every line-search trial, in order).
    callback (optional): called as callback(m + 1, obj, probe) after each
    update, for recording iterates; it must not modify them."""
    x = [np.array(obj0, dtype=np.complex128)]
    if update_probe:
        x.append(np.array(probe0, dtype=np.complex128))
    probe_fixed = np.asarray(probe0, dtype=np.complex128)

    def unpack(blocks):
        return blocks[0], (blocks[1] if update_probe else probe_fixed)

    trace = []
    g_old = None
    eta = None
    restart = True
    for m in range(iters):
        o, p = unpack(x)
        res = grad(o, p, pos, d, eps, want_probe=update_probe, estimator=estimator)
        g_new = [res["grad_obj"]] + ([res["grad_probe"]] if update_probe else [])
        phi_m = res["phi"]
        if target_phi is not None and phi_m <= target_phi:
            break
        # DIR stage
        if restart or eta is None:
            beta, restarted = 0.0, True
        else:
            beta, restarted = dai_yuan_beta(g_new, g_old, eta)
        eta = [-gn + beta * e for gn, e in zip(g_new, eta)] if not restarted \
            else [-gn for gn in g_new]

        # LS stage
        def phi_of_gamma(gamma):
            oo, pp = unpack([b + gamma * e for b, e in zip(x, eta)])
            return minfunc(oo, pp, pos, d, eps, estimator)[0]

        trial_values = []
        gamma, trials, accepted = line_search(phi_of_gamma, phi_m, gamma0, tau, t, lmax, trial_values)
        # Update stage
        x = [b + gamma * e for b, e in zip(x, eta)]
        step = gamma * math.sqrt(sum(inner(e, e).real for e in eta))
        trace.append({"phi": phi_m, "f": res["f"], "gamma": gamma,
                      "halvings": trials, "beta": beta, "step_norm": step,
                      "restarted": bool(restarted), "trial_phis": trial_values})
        g_old = g_new
        restart = not accepted
        if callback is not None:
            callback(m + 1, *unpack(x))
    o, p = unpack(x)
    return o, p, trace


# ------------------------------------------------------ GD (Eq. update2)
def gd_solve(obj0, probe0, pos, d, iters: int, gamma: float, eps: float = EPS,
             update_probe: bool = False, estimator: str = "ml"):
    """Gradient-descent solver of Eq. update2: psi_{m+1} = psi_m - gamma
    grad F(psi_m) with a constant step gamma (the paper's slower baseline).
    Joint mode also steps the probe with the same gamma along its gradient.
    Returns (obj, probe, trace) with one row per iteration: phi, f (at
    psi_m) and step_norm = gamma ||grad F(psi_m)||."""
    o = np.array(obj0, dtype=np.complex128)
    p = np.array(probe0, dtype=np.complex128)
    trace = []
    for _ in range(iters):
        res = grad(o, p, pos, d, eps, want_probe=update_probe, estimator=estimator)
        g2 = inner(res["grad_obj"], res["grad_obj"]).real
        o = o - gamma * res["grad_obj"]
        if update_probe:
            g2 += inner(res["grad_probe"], res["grad_probe"]).real
            p = p - gamma * res["grad_probe"]
        trace.append({"phi": res["phi"], "f": res["f"], "step_norm": gamma * math.sqrt(g2)})
    return o, p, trace


# ---------------------------------------------------------- comparison helper
def align_phase(rec: np.ndarray, ref: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Remove the unobservable global phase: rec * exp(i phi*) with
    phi* = arg sum_mask conj(rec) ref."""
    s = np.vdot(rec[mask], ref[mask])
    return rec * np.exp(1j * np.angle(s))
