"""Shared helpers for the GPU parity tests (imported by tests only)."""
import numpy as np


def require_gpu():
    import pytest
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_13965_amd import binding
    binding.lib()      # raises if the HIP library is missing: no silent fallback
    return binding


def sample_indices(n, k, seed=0):
    """First 64, last 64 (ragged tail) and k random indices of [0, n)."""
    g = np.random.default_rng(seed)
    idx = np.unique(np.concatenate([np.arange(min(64, n)), np.arange(max(0, n - 64), n),
                                    g.integers(0, n, size=k)]))
    return idx


def drop_rejected(g, max_frac=1e-4):
    """Exit records without the samples the decoder rejected (face -1: a network state outside
    the decodable range), after checking that they are rare."""
    ok = np.asarray(g["face"]) >= 0
    assert (~ok).mean() <= max_frac, f"{(~ok).sum()} rejected samples"
    return {k: np.asarray(v)[ok] for k, v in g.items()}


def face_threshold_margin(a4):
    """Distance of a4 from the nearest face-decoding threshold (-1, 0, 1)."""
    return np.min(np.abs(np.asarray(a4)[:, None] - np.array([-1.0, 0.0, 1.0])[None, :]), axis=1)
