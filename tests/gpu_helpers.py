"""Helpers for the GPU parity tests (host side only)."""
import numpy as np
import torch


def dev():
    return torch.device("cuda:0")


def to_dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=dev(), dtype=dtype)


def round_to_format(x: np.ndarray, sig_bits: int, min_normal_exp: int) -> np.ndarray:
    """Round float64 values to nearest-even in a binary format with `sig_bits`
    significant bits (8 for BF16, 11 for FP16) and smallest normal exponent
    `min_normal_exp` (-126 for BF16, -14 for FP16), denormals included.
    Exact: the scaled value x / ulp is an integer-spaced float64, and np.rint
    rounds half to even.  Inputs here are finite and far from overflow."""
    x = np.asarray(x, dtype=np.float64)
    ax = np.abs(x)
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.where(ax > 0, ax, 1.0)))
    # guard log2 rounding at exact powers of two
    e = np.where(np.ldexp(1.0, e.astype(np.int64)) > ax, e - 1, e)
    e = np.where(np.ldexp(1.0, (e + 1).astype(np.int64)) <= ax, e + 1, e)
    e = np.maximum(e, min_normal_exp)
    ulp = np.ldexp(1.0, (e - (sig_bits - 1)).astype(np.int64))
    return np.where(ax > 0, np.rint(x / ulp) * ulp, x)


def bf16_rne(x):
    return round_to_format(x, 8, -126)


def fp16_rne(x):
    return round_to_format(x, 11, -14)


def check_fp64_beta(tag, got, oracle_beta, closed_form, kappa_r, bar=1e-10):
    """The FP64 bar on beta with the conditioning rule: beta within `bar` of
    the oracle's (relative, Frobenius), unless the problem is
    conditioning-limited (kappa_r^2 2^-53 above the bar: two correct FP64
    normal-equation solvers may then differ by more than the bar).  Such a
    case is reported with kappa_r and its distance to the duplicated-column
    closed form (accurate to about kappa_r eps), beside the oracle's own, and
    must lie within kappa_r^2 2^-53 of that closed form.  Returns the error
    against the oracle."""
    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))
    err = rel(got, oracle_beta)
    k2e = kappa_r * kappa_r * 2.0 ** -53
    if err <= bar or k2e <= bar:
        print(f"{tag}: beta err vs oracle {err:.2e} (bar {bar:.0e}; kappa_r^2 eps {k2e:.1e})")
        assert err <= bar
        return err
    err_c, err_o = rel(got, closed_form), rel(oracle_beta, closed_form)
    print(f"{tag}: conditioning-limited (kappa_r {kappa_r:.0f}, kappa_r^2 eps {k2e:.1e}): vs oracle "
          f"{err:.2e}; vs closed form: library {err_c:.2e}, oracle {err_o:.2e} (bar kappa_r^2 eps)")
    assert err_c <= k2e
    return err
