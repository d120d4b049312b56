"""Helpers shared by the GPU tests (no arithmetic of the method here)."""
import numpy as np

# Field scales for the normwise parity metric: an error is measured against
# max(max |reference|, scale), so that small derived fields (the velocity)
# are not measured relative to round-off-sized values.
SCALES = dict(f=1.0 / 36.0, q=1.0 / 3.0, rho=1.0, u=1.0 / np.sqrt(3.0), F=1e-3, S=1.0 / 3.0)


def rel_err(a, b, scale):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), scale))


def lattice_name(lat):
    return "D2Q9" if lat == 0 else "D3Q19"


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a visible GPU")
