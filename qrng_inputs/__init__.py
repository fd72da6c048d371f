"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no arithmetic of the method (no hashing, no entropy
estimate): it only draws the raw ADC stream and the uniform seeds, so the
oracle and the HIP path can be fed identical bytes.

Recipe (the paper's raw data files are not available; these stand in):

* ADC samples: N = 8 bits per sample, u = clip(rint(mu + sigma z), 0, 255)
  with z ~ N(0, 1) from numpy's PCG64 ``default_rng(seed)``; rint rounds half
  to even.  Mean 128, sigma 20 unless stated.
* Raw bits: sample t contributes bits 8t..8t+7, LSB first, so the uint8 sample
  buffer viewed as little-endian uint64 words *is* the packed raw block.
* Toeplitz seeds: ``default_rng(seed).integers(0, 2**64, ceil(L/64))`` words.
  Bits at positions >= L are left random on purpose: consumers must ignore
  them.
* Adversarial ADC stream (the attacked detector of Sec. II.B): intensity
  I ~ N(0, 1), photodiode gain alpha(I) = alpha_e (1 - I / (beta_e I_max))
  with alpha_e = 0.99, beta_e = 2, I_max = 5, output V' = alpha(I) I,
  digitised by an N-bit ADC over [-5, 5): code floor((V' + 5) / (10 / 2^N)),
  clipped to [0, 2^N - 1] (the end codes take the tails).
* Named workloads: ``config(k)`` returns the fixed seeds and sizes of the
  five workloads (single block n = 2^17; single block n = 2^23; block-length
  sweep over a 2^30-bit stream; 4096 uneven batched blocks; serving loop).
"""
from __future__ import annotations

import math

import numpy as np

SAMPLE_BITS = 8

# Fixed generator seeds, one per workload.
SEEDS = {
    "single_n2^17": {"adc": 20201101, "seed": 11042020},
    "single_n2^23": {"adc": 20201102, "seed": 11042021},
    "sweep_2^30": {"adc": 20201103, "seed": 11042022},
    "batched_4096": {"adc": 20201104, "seed": 11042023, "shape": 7},
    "serve": {"adc": 20201105, "seed": 11042024, "arrivals": 99},
}


def gen_adc(S: int, sigma: float = 20.0, mu: float = 128.0, seed: int = 0,
            bits: int = SAMPLE_BITS) -> np.ndarray:
    """S Gaussian ADC samples as uint8 (clipped to [0, 2^bits - 1])."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(S)
    u = np.clip(np.rint(mu + sigma * z), 0, (1 << bits) - 1)
    return u.astype(np.uint8)


def gen_attack(S: int, bits: int = 5, seed: int = 0, alpha_e: float = 0.99,
               beta_e: float = 2.0, i_max: float = 5.0) -> np.ndarray:
    """S samples of the attacked detector output V' = alpha(I) I as N-bit
    ADC codes over [-5, 5) (uint8)."""
    rng = np.random.default_rng(seed)
    i = rng.standard_normal(S)
    v = alpha_e * (1.0 - i / (beta_e * i_max)) * i
    w = 10.0 / (1 << bits)
    return np.clip(np.floor((v + 5.0) / w), 0, (1 << bits) - 1).astype(np.uint8)


def gen_seed_words(L: int, seed: int = 0) -> np.ndarray:
    """ceil(L/64) uniform uint64 words (bits >= L left random)."""
    rng = np.random.default_rng(seed)
    nw = max((L + 63) // 64, 1)
    return rng.integers(0, 2 ** 64, nw, dtype=np.uint64)


def gen_bits(nbits: int, seed: int = 0) -> np.ndarray:
    """nbits uniform bits as packed uint64 words (tail bits random too)."""
    return gen_seed_words(nbits, seed)


def samples_as_words(samples: np.ndarray) -> np.ndarray:
    """View a uint8 sample buffer (length a multiple of 8) as uint64 words."""
    assert len(samples) % 8 == 0
    return np.ascontiguousarray(samples).view("<u8")


def config(k: int) -> dict:
    """Sizes and seeds of the named workloads (k = 0..4)."""
    if k == 0:
        s = SEEDS["single_n2^17"]
        return {"name": "single_n2^17", "S": 16384, "sigma": 20.0, "n": 131072,
                "m_expected": 81920, "adc_seed": s["adc"], "seed_seed": s["seed"]}
    if k == 1:
        s = SEEDS["single_n2^23"]
        n = 1 << 23
        return {"name": "single_n2^23", "S": 1 << 20, "sigma": 20.0, "n": n,
                "m_expected": (n * 5) // 8, "adc_seed": s["adc"],
                "seed_seed": s["seed"]}
    if k == 2:
        s = SEEDS["sweep_2^30"]
        return {"name": "sweep_2^30", "S": 1 << 27, "sigma": 20.0,
                "total_bits": 1 << 30, "block_log2": list(range(12, 25, 2)),
                "gamma_num": 5, "gamma_den": 8, "adc_seed": s["adc"],
                "seed_seed": s["seed"]}
    if k == 3:
        s = SEEDS["batched_4096"]
        return {"name": "batched_4096", "blocks": 4096, "group": 64,
                "log2_min": 14, "log2_max": 20, "sigma_min": 8.0,
                "sigma_max": 40.0, "adc_seed": s["adc"], "seed_seed": s["seed"],
                "shape_seed": s["shape"]}
    if k == 4:
        s = SEEDS["serve"]
        return {"name": "serve", "window_samples": 1 << 24, "sigma": 20.0,
                "rates": [1000, 2000, 5000, 10000, 20000, 50000],
                "r_log2_min": 8, "r_log2_max": 24, "adc_seed": s["adc"],
                "seed_seed": s["seed"], "arrival_seed": s["arrivals"]}
    raise ValueError(k)


def batched_shapes(cfg: dict) -> dict:
    """Per-block raw lengths and sigmas of the uneven batched workload.

    n_b = 64 * floor(2^U(log2_min, log2_max) / 64); sigma_b ~ U[sigma_min,
    sigma_max]; each block's samples come from ``gen_adc`` with its own seed.
    """
    rng = np.random.default_rng(cfg["shape_seed"])
    B = cfg["blocks"]
    e = rng.uniform(cfg["log2_min"], cfg["log2_max"], B)
    n = (np.floor(2.0 ** e / 64.0).astype(np.int64) * 64)
    n = np.maximum(n, 64)
    sig = rng.uniform(cfg["sigma_min"], cfg["sigma_max"], B)
    return {"n": n, "sigma": sig}


def batched_pool(cfg: dict) -> dict:
    """Sample pool of the uneven batched workload.

    Block b draws n_b / 8 samples with ``gen_adc(sigma=sigma_b, seed=adc_seed
    + b)``; blocks are concatenated in order (n_b is a multiple of 64, so each
    block starts 8-byte aligned).  Block b uses seed group b // group, whose
    seed words are ``gen_seed_words(seed_bits, seed_seed + g)`` with
    seed_bits = 2 max(n) (enough for any m <= n).
    """
    sh = batched_shapes(cfg)
    n, sig = sh["n"], sh["sigma"]
    S = n // 8
    off = np.concatenate([[0], np.cumsum(S)[:-1]]).astype(np.int64)
    pool = np.empty(int(S.sum()), dtype=np.uint8)
    for b in range(len(n)):
        pool[off[b]:off[b] + S[b]] = gen_adc(int(S[b]), float(sig[b]), seed=cfg["adc_seed"] + b)
    group = cfg["group"]
    ngroups = (len(n) + group - 1) // group
    return {"n": n, "sigma": sig, "samples": pool, "byte_off": off,
            "seed_of": np.arange(len(n)) // group, "nseeds": ngroups,
            "seed_bits": int(2 * n.max()),
            "seed_words": lambda g: gen_seed_words(int(2 * n.max()), cfg["seed_seed"] + g)}


def poisson_arrivals(rate: float, count: int, seed: int) -> np.ndarray:
    """Arrival times (seconds) of an open-loop Poisson process."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, count))


def request_sizes(count: int, lo_log2: int, hi_log2: int, seed: int) -> np.ndarray:
    """Requested output bits, log-uniform in [2^lo, 2^hi]."""
    rng = np.random.default_rng(seed)
    return np.floor(2.0 ** rng.uniform(lo_log2, hi_log2, count)).astype(np.int64)


def log2_ceil(v: int) -> int:
    return 0 if v <= 1 else int(math.ceil(math.log2(v)))
