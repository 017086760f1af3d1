"""Seeded synthetic inputs shaped like the paper's synthetic workloads.

This module holds no arithmetic of the screening method itself (no lambda_*,
no dual point, no test): it only draws dictionaries, sparse codes, noise and
penalty ratios, so that the HIP path and the test oracle can be fed identical
arrays.

Recipes (experiments section, "Data material"):
* Gaussian dictionary: atoms drawn from N(0, I_N) and normalised to unit l2
  norm, i.e. i.i.d. uniform on the unit sphere.
* Pnoise dictionary: atoms e_1 + 0.1 * kappa * g with g ~ N(0, I_N),
  kappa ~ U(0, 1), then normalised.
* Bernoulli-Gaussian codes: each atom (or group) active with probability p,
  active coefficients i.i.d. N(0, 1); observation y = D x0 + e with the noise
  scaled to a given SNR in dB, then normalised to unit l2 norm.

Every array is float64 in memory; storage precision is applied by the caller
(`to_storage`), and the stored values define the problem instance.
"""
from __future__ import annotations

import numpy as np

DICT_SEED = 0
SIGNAL_SEED0 = 1000
LAMBDA_SEED0 = 2000
ARRIVAL_SEED = 3000


def gaussian_dictionary(N: int, K: int, seed: int = DICT_SEED) -> np.ndarray:
    """N x K, column-major (Fortran order), unit-norm Gaussian atoms."""
    rng = np.random.default_rng(seed)
    D = rng.standard_normal((K, N)).T  # column i is contiguous in memory
    D = D / np.linalg.norm(D, axis=0, keepdims=True)
    return np.asfortranarray(D)


def pnoise_dictionary(N: int, K: int, seed: int = DICT_SEED) -> np.ndarray:
    """N x K Pnoise dictionary (atoms e_1 + 0.1 kappa g, normalised)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((K, N)).T
    kappa = rng.uniform(0.0, 1.0, size=K)
    D = 0.1 * kappa[None, :] * g
    D[0, :] += 1.0
    D = D / np.linalg.norm(D, axis=0, keepdims=True)
    return np.asfortranarray(D)


def bernoulli_gaussian_code(K: int, p: float, rng: np.random.Generator,
                            group_ptr: np.ndarray | None = None) -> np.ndarray:
    """Sparse code x0: atoms (or whole contiguous groups) active with probability p."""
    x0 = np.zeros(K)
    if group_ptr is None:
        mask = rng.uniform(size=K) < p
        while not mask.any():
            mask = rng.uniform(size=K) < p
        x0[mask] = rng.standard_normal(int(mask.sum()))
    else:
        G = group_ptr.size - 1
        gm = rng.uniform(size=G) < p
        while not gm.any():
            gm = rng.uniform(size=G) < p
        for g in np.flatnonzero(gm):
            a, b = group_ptr[g], group_ptr[g + 1]
            x0[a:b] = rng.standard_normal(b - a)
    return x0


def observation(D: np.ndarray, x0: np.ndarray, rng: np.random.Generator, *,
                snr_db: float | None = 20.0, noise_std: float | None = None,
                normalize: bool = True) -> np.ndarray:
    """y = D x0 + e.  With snr_db the noise norm is exactly ||D x0|| / 10^(snr/20)."""
    s = D @ x0
    e = rng.standard_normal(D.shape[0])
    if snr_db is not None:
        e *= np.linalg.norm(s) / (np.linalg.norm(e) * 10.0 ** (snr_db / 20.0))
    elif noise_std is not None:
        e *= noise_std
    else:
        e[:] = 0.0
    y = s + e
    if normalize:
        y = y / np.linalg.norm(y)
    return y


def contiguous_groups(K: int, size: int) -> np.ndarray:
    """CSR offsets of a partition of range(K) into contiguous groups of `size` atoms."""
    assert K % size == 0
    return np.arange(0, K + 1, size, dtype=np.int64)


def lambda_ratios(B: int, lo: float = 0.1, hi: float = 0.9, seed: int = LAMBDA_SEED0) -> np.ndarray:
    """Per-signal lambda / lambda_* drawn uniformly in [lo, hi]."""
    return np.random.default_rng(seed).uniform(lo, hi, size=B)


# ---------------------------------------------------------------------------
# Storage precision
# ---------------------------------------------------------------------------

def round_bf16(a: np.ndarray) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even); returns float32."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).reshape(f.shape)
    return np.asarray(out, order="F") if np.isfortran(a) else out


def bf16_bits(a: np.ndarray) -> np.ndarray:
    """uint16 bit patterns of round_bf16(a) (same memory order as the input)."""
    r = round_bf16(a)
    order = "F" if np.isfortran(r) else "C"
    return (np.asarray(r, order=order).view(np.uint32) >> 16).astype(np.uint16)


def to_storage(a: np.ndarray, dtype: str) -> np.ndarray:
    """Values of `a` as stored at precision dtype ('f64', 'f32' or 'bf16'), widened to float64."""
    if dtype == "f64":
        return np.asarray(a, dtype=np.float64)
    if dtype == "f32":
        return np.asarray(a, dtype=np.float32).astype(np.float64)
    if dtype == "bf16":
        return round_bf16(a).astype(np.float64)
    raise ValueError(dtype)


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

def lasso_small_fp64(seed: int = DICT_SEED):
    """D 100x500 Gaussian, x0 Bernoulli(0.05)-Gaussian, y = D x0 + 0.01 N(0,1) (not
    normalised), lambda = 0.5 lambda_*; ISTA + dynamic SAFE for 500 iterations in FP64."""
    D = gaussian_dictionary(100, 500, seed)
    rng = np.random.default_rng(SIGNAL_SEED0)
    x0 = bernoulli_gaussian_code(500, 0.05, rng)
    y = observation(D, x0, rng, snr_db=None, noise_std=0.01, normalize=False)
    return dict(D=D, y=y, x0=x0, lam_ratio=0.5, rule="ista", test="safe", max_iter=500,
                gap_tol=0.0, dtype="f64")


def lasso_signal(D: np.ndarray, j: int, p: float = 0.02, snr_db: float = 20.0):
    """Signal j of the Lasso workloads: Bernoulli(p)-Gaussian code, 20 dB noise, unit y."""
    rng = np.random.default_rng(SIGNAL_SEED0 + j)
    x0 = bernoulli_gaussian_code(D.shape[1], p, rng)
    return observation(D, x0, rng, snr_db=snr_db), x0


def group_signal(D: np.ndarray, group_ptr: np.ndarray, j: int, p: float = 0.02,
                 snr_db: float = 20.0):
    """Signal j of the Group-Lasso workloads: active groups Bernoulli(p), Gaussian
    coefficients, 20 dB noise, unit y."""
    rng = np.random.default_rng(SIGNAL_SEED0 + j)
    x0 = bernoulli_gaussian_code(D.shape[1], p, rng, group_ptr)
    return observation(D, x0, rng, snr_db=snr_db), x0


def atom_like_observation(N: int, j: int, kind: str = "gaussian") -> np.ndarray:
    """Observation j of the Lasso experiments, drawn from the same distribution as the atoms
    ("Data material"): uniform on the unit sphere (Gaussian), or e_1 + 0.1 kappa g with
    kappa ~ U(0, 1) (Pnoise); normalised."""
    rng = np.random.default_rng(SIGNAL_SEED0 + j)
    v = rng.standard_normal(N)
    if kind == "pnoise":
        v = 0.1 * rng.uniform(0.0, 1.0) * v
        v[0] += 1.0
    elif kind != "gaussian":
        raise ValueError(kind)
    return v / np.linalg.norm(v)


LASSO_SWEEP = (0.1, 0.3, 0.5, 0.7, 0.9)
GROUP_SWEEP = (0.3, 0.7)
