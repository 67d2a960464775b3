"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import numpy as np

# Per-image relative L2 bound of the FP32 GPU path against the FP64 oracle on
# the same inputs and the same random stream.  FP32 rounding in the FFTs and
# updates drifts by ~1e-6 per image after 1000 sweeps (measured on CPU with an
# FP32 emulation of the sweep); 1e-4 leaves a wide margin.
REL_TOL = 1e-4


def rel(a, b):
    """Relative L2 distance (complex arrays: over real and imaginary parts);
    +inf if either side holds a NaN or Inf (so a max() over cases or a <
    comparison can never hide one)."""
    a, b = np.asarray(a), np.asarray(b)
    if np.iscomplexobj(a) or np.iscomplexobj(b):
        a = np.concatenate([np.real(a).ravel(), np.imag(a).ravel()])
        b = np.concatenate([np.real(b).ravel(), np.imag(b).ravel()])
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if not (np.all(np.isfinite(a)) and np.all(np.isfinite(b))):
        return float("inf")
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def banner(msg):
    print(f"\n[gpu] {msg}", flush=True)
