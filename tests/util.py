"""Shared helpers for the tests (no method arithmetic here)."""
import numpy as np

# Textbook cold-plasma dispersion constant (us MHz^2 cm^3 / pc), used only to
# synthesise dispersed test pulses.
K_DM_US = 4.148808e9


def arrival_law(dm, f_ref):
    """Physical arrival time (us) of frequency f relative to f_ref."""
    return lambda f: K_DM_US * dm * (1.0 / (f * f) - 1.0 / (f_ref * f_ref))


def rel_l2(got, want):
    got = np.asarray(got, dtype=np.complex128 if np.iscomplexobj(got) else np.float64)
    want = np.asarray(want, dtype=got.dtype)
    den = np.linalg.norm(want.ravel())
    num = np.linalg.norm((got - want).ravel())
    return num / den if den > 0 else num


def gpu():
    import torch
    return torch.device("cuda:0")


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(gpu())


def flush(msg):
    print(msg, flush=True)
