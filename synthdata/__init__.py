"""Seeded synthetic workloads shaped like the paper's benchmark data.

This module only draws random numbers and shapes them into point sets; it holds
none of the search method's arithmetic (no projection fit, no distances, no
pruning), so both the FP64 oracle and the GPU library may take their inputs
from it without sharing any of the method.

The paper evaluates on public descriptor / embedding collections (Sec. VII-A,
Table I). None of them is available here, so every workload below is a
synthetic stand-in with the dimensionality, size and kind of spectrum of one
of them:

* ``gauss``   -- zero-mean Gaussian, eigen-spectrum lambda_i = 1/i under a Haar
  rotation (a clean case for the Gaussian error model of Sec. IV-B).
* ``sift``    -- 128-d, integer valued 0..255 (SIFT-like image descriptors,
  Table I), a mixture of anisotropic Gaussians, clipped and rounded.
* ``gist``    -- 960-d (GIST's dimensionality, Table I), mixture of Gaussians
  with a power-law spectrum lambda_i = i^-1.2.
* ``embed``   -- unit-normalised embeddings (power-law spectrum), used for the
  768-d batched workload and the 256-d serving workload.

Random streams: seed = 1000 * config_id + stream, with streams base 1,
queries 2, calibration 3, validation 4, rotation 5, mixture parameters 6.
All generators are numpy's PCG64 (``numpy.random.default_rng``).
"""
from __future__ import annotations

import numpy as np

STREAM_BASE, STREAM_QUERY, STREAM_CALIB, STREAM_VAL, STREAM_ROT, STREAM_MIX = 1, 2, 3, 4, 5, 6


def haar_rotation(D: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of a Gaussian matrix with the
    signs of diag(R) folded into Q (Mezzadri, 'How to generate random matrices
    from the classical compact groups', 2007)."""
    g = rng.standard_normal((D, D))
    q, r = np.linalg.qr(g)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :]


def gauss_points(n: int, D: int, seed: int, rot: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """x = Q (sqrt(lambda) * z), z ~ N(0, I): zero-mean Gaussian with covariance
    Q diag(lambda) Q^T.  Returned as float32, row-major (n, D)."""
    rng = np.random.default_rng(seed)
    out = np.empty((n, D), dtype=np.float32)
    sl = np.sqrt(lam)
    chunk = 1 << 16
    for s in range(0, n, chunk):
        z = rng.standard_normal((min(chunk, n - s), D))
        out[s:s + z.shape[0]] = (z * sl[None, :]) @ rot.T
    return out


class Mixture:
    """Mixture of anisotropic Gaussians sharing one global rotation Q.

    Component means: centre + a * Q (sqrt(lambda) * z_c).  Within component c:
    b * Q (sqrt(lambda * j_c) * z), with a per-component, per-dimension jitter
    j_c ~ LogNormal(0, 0.5^2), so every component has its own anisotropy.
    """

    def __init__(self, D: int, n_comp: int, lam: np.ndarray, centre: float, mean_std: float,
                 within_std: float, seed_rot: int, seed_mix: int):
        self.D, self.n_comp = D, n_comp
        self.rot = haar_rotation(D, np.random.default_rng(seed_rot))
        rng = np.random.default_rng(seed_mix)
        norm = np.sqrt(lam.sum() / D)            # per-coordinate std of Q(sqrt(lam) z)
        a = mean_std / norm
        b = within_std / norm
        zc = rng.standard_normal((n_comp, D))
        self.means = centre + a * ((zc * np.sqrt(lam)[None, :]) @ self.rot.T)
        jitter = rng.lognormal(0.0, 0.5, size=(n_comp, D))
        self.scales = b * np.sqrt(lam[None, :] * jitter)   # in the rotated frame

    def sample(self, n: int, seed: int, post=None, dtype=np.float64) -> np.ndarray:
        """n points; `post` (optional) maps every FP64 chunk before it is stored as `dtype`
        (the random draws do not depend on either)."""
        rng = np.random.default_rng(seed)
        comp = rng.integers(0, self.n_comp, size=n)
        out = np.empty((n, self.D), dtype=dtype)
        chunk = 1 << 16
        for s in range(0, n, chunk):
            c = comp[s:s + chunk]
            z = rng.standard_normal((c.shape[0], self.D))
            x = self.means[c] + (z * self.scales[c]) @ self.rot.T
            out[s:s + c.shape[0]] = post(x) if post is not None else x
        return out


def _power_spectrum(D: int, expo: float) -> np.ndarray:
    return np.arange(1, D + 1, dtype=np.float64) ** (-expo)


# name -> (config id, D, n_base, n_query, n_calib, n_val, kind, extra)
WORKLOADS = {
    # 10,000 base + 100 queries, D=128, lambda_i = 1/i, Haar rotation
    "gauss128": dict(cfg=1, D=128, n=10_000, nq=100, n_calib=1_000, n_val=1_000, kind="gauss", expo=1.0),
    # 1M x 128, integers 0..255, 1,024 anisotropic components, 10,000 queries
    "sift1m": dict(cfg=2, D=128, n=1_000_000, nq=10_000, n_calib=1_000, n_val=1_000, kind="sift",
                   comps=1024, expo=1.0),
    # 1M x 960, 256 components, lambda_i = i^-1.2, 1,000-query batches
    "gist1m": dict(cfg=3, D=960, n=1_000_000, nq=1_000, n_calib=1_000, n_val=1_000, kind="gist",
                   comps=256, expo=1.2),
    # 2M x 768 unit-normalised, 512 clusters, 4,096 queries per launch
    "embed768": dict(cfg=4, D=768, n=2_000_000, nq=4_096, n_calib=1_000, n_val=1_000, kind="embed",
                     comps=512, expo=1.0),
    # 5M x 256 unit-normalised, 1,024 clusters (serving)
    "embed256": dict(cfg=5, D=256, n=5_000_000, nq=4_096, n_calib=1_000, n_val=1_000, kind="embed",
                     comps=1024, expo=1.0),
}


def make_workload(name: str, n: int | None = None, nq: int | None = None,
                  n_calib: int | None = None, n_val: int | None = None,
                  spread: tuple | None = None) -> dict:
    """Build a workload.  Sizes default to the full configuration; smaller
    sizes draw from the same distribution (same rotation and mixture), so a
    reduced case is a prefix-free sample of the same data source.

    Returns dict(base, queries, calib, val) as float32 C-contiguous arrays plus
    the recipe (``spec``) and, for the Gaussian case, the true spectrum and
    rotation (``lam``, ``rot``) for closed-form checks.  ``spread`` overrides the
    mixture's (between-component, within-component) per-coordinate std.
    """
    spec = dict(WORKLOADS[name])
    n = spec["n"] if n is None else n
    nq = spec["nq"] if nq is None else nq
    n_calib = spec["n_calib"] if n_calib is None else n_calib
    n_val = spec["n_val"] if n_val is None else n_val
    cfg, D, kind = spec["cfg"], spec["D"], spec["kind"]
    sd = lambda stream: 1000 * cfg + stream
    out = dict(spec=spec, name=name)
    if kind == "gauss":
        lam = _power_spectrum(D, spec["expo"])
        rot = haar_rotation(D, np.random.default_rng(sd(STREAM_ROT)))
        out["lam"], out["rot"] = lam, rot
        gen = lambda cnt, stream: gauss_points(cnt, D, sd(stream), rot, lam)
    else:
        lam = _power_spectrum(D, spec["expo"])
        if kind == "sift":
            ms, ws = spread or (21.0, 24.0)
            mix = Mixture(D, spec["comps"], lam, centre=127.5, mean_std=ms, within_std=ws,
                          seed_rot=sd(STREAM_ROT), seed_mix=sd(STREAM_MIX))

            def gen(cnt, stream):   # clip to [0, 255], round half-even
                return mix.sample(cnt, sd(stream), post=lambda x: np.rint(np.clip(x, 0.0, 255.0)),
                                  dtype=np.float32)
        elif kind == "gist":
            mix = Mixture(D, spec["comps"], lam, centre=0.0, mean_std=0.6, within_std=0.4,
                          seed_rot=sd(STREAM_ROT), seed_mix=sd(STREAM_MIX))
            gen = lambda cnt, stream: mix.sample(cnt, sd(stream), dtype=np.float32)
        elif kind == "embed":
            mix = Mixture(D, spec["comps"], lam, centre=0.0, mean_std=0.6, within_std=0.4,
                          seed_rot=sd(STREAM_ROT), seed_mix=sd(STREAM_MIX))

            def gen(cnt, stream):   # unit-normalised after sampling
                return mix.sample(cnt, sd(stream), post=lambda x: x / np.linalg.norm(x, axis=1, keepdims=True),
                                  dtype=np.float32)
        else:
            raise ValueError(kind)
    out["base"] = np.ascontiguousarray(gen(n, STREAM_BASE))
    out["queries"] = np.ascontiguousarray(gen(nq, STREAM_QUERY))
    out["calib"] = np.ascontiguousarray(gen(n_calib, STREAM_CALIB)) if n_calib else np.zeros((0, D), np.float32)
    out["val"] = np.ascontiguousarray(gen(n_val, STREAM_VAL)) if n_val else np.zeros((0, D), np.float32)
    return out


def uneven_requests(nq: int, seed: int, nprobe_lo: int, nprobe_hi: int, k_choices) -> tuple:
    """Per-query (K, nprobe) draws for the batched uneven-probe workload:
    nprobe ~ U{lo..hi}, K uniform over ``k_choices``."""
    rng = np.random.default_rng(seed)
    nprobe = rng.integers(nprobe_lo, nprobe_hi + 1, size=nq).astype(np.int32)
    k = np.asarray(k_choices, dtype=np.int32)[rng.integers(0, len(k_choices), size=nq)]
    return k, nprobe


STREAM_OOD = 11   # streams 11, 12, 13: out-of-distribution queries, calibration, validation


def ood_queries(name: str, n: int, stream: int = STREAM_OOD, within_scale: float = 2.0) -> np.ndarray:
    """Queries from a shifted distribution (out-of-distribution for an index fitted on the
    workload): for the mixtures, the same component means with every within-component scale
    multiplied by ``within_scale`` (noisier queries, same post-processing); for the Gaussian
    case, another Haar rotation and the flatter spectrum lambda_i = i^-0.5 at the same total
    variance."""
    spec = dict(WORKLOADS[name])
    cfg, D, kind = spec["cfg"], spec["D"], spec["kind"]
    sd = 1000 * cfg + stream
    lam = _power_spectrum(D, spec["expo"])
    if kind == "gauss":
        rot2 = haar_rotation(D, np.random.default_rng(1000 * cfg + STREAM_ROT + 10))
        lam2 = _power_spectrum(D, 0.5)
        lam2 *= lam.sum() / lam2.sum()
        return np.ascontiguousarray(gauss_points(n, D, sd, rot2, lam2))
    centre, ms, ws = {"sift": (127.5, 21.0, 24.0), "gist": (0.0, 0.6, 0.4), "embed": (0.0, 0.6, 0.4)}[kind]
    mix = Mixture(D, spec["comps"], lam, centre=centre, mean_std=ms, within_std=ws,
                  seed_rot=1000 * cfg + STREAM_ROT, seed_mix=1000 * cfg + STREAM_MIX)
    mix.scales = mix.scales * within_scale
    if kind == "sift":
        post = lambda x: np.rint(np.clip(x, 0.0, 255.0))
    elif kind == "embed":
        post = lambda x: x / np.linalg.norm(x, axis=1, keepdims=True)
    else:
        post = None
    return np.ascontiguousarray(mix.sample(n, sd, post=post, dtype=np.float32))
