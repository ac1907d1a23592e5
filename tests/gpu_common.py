"""Comparison helpers shared by the GPU parity tests.

The bar: relative L2 over the field <= 1e-12 in FP64 and <= 1e-5 in FP32,
and the same bound per element, max |got - ref| / max |ref|, so that an error
confined to a few nodes (a line end, a strip end, a tile seam) is not diluted
by the size of the field.  Every comparison prints both measures.
"""
import numpy as np

TOL = {"f64": 1e-12, "f32": 1e-5}


def rel(a, b):
    """Relative L2 error of a against b (absolute when b is zero)."""
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def elem(a, b):
    """Largest error of a single element, relative to the largest |b|."""
    mb = float(np.abs(b).max()) if np.size(b) else 0.0
    return float(np.abs(a - b).max() / (mb if mb > 0 else 1.0)) if np.size(b) else 0.0


def check(name, got, ref, dtype, tol=None):
    """Assert relative L2 and per-element error <= tol (default: the bar of dtype)."""
    t = TOL[dtype] if tol is None else tol
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    e, m = rel(got, ref), elem(got, ref)
    print("%-52s %s rel L2 = %.3e  max elem = %.3e" % (name, dtype, e, m))
    if m > t and got.size:
        i = int(np.abs(got - ref).argmax())
        print("    largest error at index %s: got %.17g ref %.17g (max |ref| %.6g)"
              % (np.unravel_index(i, got.shape), got.ravel()[i], ref.ravel()[i], np.abs(ref).max()))
    assert np.isfinite(got).all(), name
    assert e <= t, (name, "rel L2", e)
    assert m <= t, (name, "max elem", m)
    return e


def dev(torch, a, dtype):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to(device="cuda", dtype=torch.float64 if dtype == "f64" else torch.float32)


def host(t):
    return t.double().cpu().numpy()
