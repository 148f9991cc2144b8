"""Helpers shared by the GPU tests: device tensors in the library's layout."""
import numpy as np


def to_dev_soa(x: np.ndarray):
    """[n][d] host array -> [d][n] float64 cuda tensor."""
    import torch

    return torch.from_numpy(np.ascontiguousarray(x.T)).to("cuda")


def rel_err(a, b, floor=0.0):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.maximum(np.abs(b), floor)
    out = np.zeros_like(a)
    nz = den > 0
    out[nz] = np.abs(a[nz] - b[nz]) / den[nz]
    out[~nz] = np.abs(a[~nz] - b[~nz])
    return out


def assert_close(got, ref, rtol, floor_frac=1e-14):
    """|got - ref| <= rtol |ref| + floor_frac max|ref| element by element.

    The absolute floor (a fraction of the largest value) covers events whose
    value sits on a cancellation -- the PDF interpolant crossing zero near
    x -> 1, or x within one rounding of the last knot where one side gives 0
    and the other ~1e-38 -- where two FP64 evaluations differ by rounding
    relative to the scale of the integrand rather than to the value itself.
    """
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    atol = floor_frac * float(np.max(np.abs(ref)))
    bad = np.abs(got - ref) > rtol * np.abs(ref) + atol
    assert not bad.any(), (int(bad.sum()), np.flatnonzero(bad)[:5], got[bad][:5], ref[bad][:5])


def bf16_round(a) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as float64:
    parameters given in this form are exact in the kernels' BF16 copies."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def cosine_rel_l2(got, ref):
    """(cosine similarity, |got - ref| / |ref|) of two flattened arrays."""
    g = np.asarray(got, dtype=np.float64).ravel()
    r = np.asarray(ref, dtype=np.float64).ravel()
    cos = float(g @ r / (np.linalg.norm(g) * np.linalg.norm(r)))
    return cos, float(np.linalg.norm(g - r) / np.linalg.norm(r))
