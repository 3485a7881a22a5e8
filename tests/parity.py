"""Error metrics shared by the GPU parity tests (tolerances are in the tests)."""
import numpy as np


def wrap(x):
    """Map angles to (-pi, pi]."""
    return np.angle(np.exp(1j * np.asarray(x)))


def log_rho_err(got, ref):
    """max_b (|dRe| + |wrap(dIm)|) / max(1, max |ref|): complex log-amplitudes."""
    got = np.asarray(got)
    g = got[..., 0] + 1j * got[..., 1] if got.ndim >= 2 and got.shape[-1] == 2 and not np.iscomplexobj(got) else got
    d = g - ref
    return float(np.max(np.abs(np.real(d)) + np.abs(wrap(np.imag(d)))) / max(1.0, float(np.max(np.abs(ref)))))


def rel_l2(got, ref):
    return float(np.linalg.norm(np.asarray(got) - np.asarray(ref)) / max(np.linalg.norm(ref), 1e-300))
