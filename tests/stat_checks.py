"""Statistical comparison shared by the GPU parity tests (not a test module)."""
import numpy as np


def compare_3sigma(a, ea, b, eb, frac=0.01):
    """Reading of 'within 3 sigma': |a - b| <= 3 sqrt(ea^2 + eb^2) per point, at
    most `frac` of the points beyond, none beyond 5 sigma.  Returns the z-scores."""
    z = np.abs(np.asarray(a) - np.asarray(b)) / np.sqrt(np.asarray(ea) ** 2 + np.asarray(eb) ** 2)
    assert np.all(np.isfinite(z)), z
    assert z.max() < 5.0, (z.max(), int(np.argmax(z)))
    assert np.mean(z > 3.0) <= frac, (np.mean(z > 3.0), np.sort(z)[-5:])
    return z


def read_fixture(path):
    """Rows of a tests/golden text fixture: {tag: [row fields as floats]} (comments skipped)."""
    out = {}
    with open(path) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            tag, *rest = line.split()
            out.setdefault(tag, []).append([float(x) for x in rest])
    return out
