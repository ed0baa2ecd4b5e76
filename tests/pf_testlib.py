"""Helpers shared by the GPU parity tests: tolerances and layout conversions.

Tolerances: states and log-weights must agree within 1e-5 relative, measured
as |g - o| <= 1e-5 * max(|o|, floor) per element (floor 1 for Lorenz states
and log-weights, 0.1 for FH-N v/w), so that values near zero do not demand
an absolute accuracy below FP32 resolution.  Ancestors must be identical
except for slots whose uniform lies within 1e-6 (relative to C_{N-1}) of a
CDF value.
"""
import numpy as np

REL = 1e-5
BAND = 1e-6


def rel_close(g, o, floor=1.0, rel=REL):
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    both_inf = np.isinf(g) & np.isinf(o) & (np.sign(g) == np.sign(o))
    err = np.abs(g - o)
    tol = rel * np.maximum(np.abs(o), floor)
    ok = both_inf | (err <= tol)
    return ok


def assert_rel_close(g, o, floor=1.0, rel=REL, what="values"):
    ok = rel_close(g, o, floor, rel)
    if not ok.all():
        g = np.asarray(g, dtype=np.float64)
        o = np.asarray(o, dtype=np.float64)
        bad = np.argwhere(~ok)
        i = tuple(bad[0])
        raise AssertionError(
            f"{what}: {(~ok).sum()} of {ok.size} outside rel {rel} (floor {floor}); "
            f"first at {i}: gpu={g[i]!r} oracle={o[i]!r}; max abs err "
            f"{np.nanmax(np.abs(g - o)[np.isfinite(g - o)]) if np.isfinite(g - o).any() else 'n/a'}")


def band_mask(C, U):
    """True where U_k * C_{N-1} lies within BAND * C_{N-1} of some C_i."""
    C = np.asarray(C, dtype=np.float64)
    v = np.asarray(U, dtype=np.float64) * C[-1]
    pos = np.searchsorted(C, v)
    lo = np.clip(pos - 1, 0, C.size - 1)
    hi = np.clip(pos, 0, C.size - 1)
    d = np.minimum(np.abs(C[lo] - v), np.abs(C[hi] - v))
    return d < BAND * C[-1]


def vec_to_oracle(x):
    """[M, D, N] (device layout of vector models) -> [M, N, D]."""
    return np.ascontiguousarray(np.transpose(np.asarray(x), (0, 2, 1)))


def oracle_to_vec(x):
    """[M, N, D] -> [M, D, N]."""
    return np.ascontiguousarray(np.transpose(np.asarray(x), (0, 2, 1)))
