"""Shared helpers for the GPU parity tests (GPU path vs the FP64 oracle)."""
import numpy as np

from oracle import oracle as O


def rel_l2(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    den = np.linalg.norm(want)
    return float(np.linalg.norm(got - want) / den) if den > 0 else float(np.linalg.norm(got))


def field_rel_l2(gpu_fields, orc_fields):
    """max over E and H of ||gpu - oracle||_2 / ||oracle||_2 (all cells)."""
    e = rel_l2(gpu_fields[:3], orc_fields[:3])
    h = rel_l2(gpu_fields[3:], orc_fields[3:])
    return max(e, h)


def run_oracle(cfg, steps):
    sim = O.OracleSim(cfg, max_steps=steps)
    sim.step(steps)
    return sim


def run_gpu(cfg, steps, tuning=None, chunks=None):
    import torch
    from paper_0802_3775_amd import fdtd as F
    plan = F.Plan(cfg, max_steps=steps, tuning=tuning)
    if chunks:
        for c in chunks:
            plan.step(c)
    else:
        plan.step(steps)
    torch.cuda.synchronize()
    return plan


def pec_clean(fields, periodic):
    """Zero the E components that sit on PEC walls (tangential at index 0)."""
    for c, axes in ((0, (1, 2)), (1, (0, 2)), (2, (0, 1))):
        for a in axes:
            if not periodic[a]:
                sl = [slice(None)] * 3
                sl[2 - a] = 0
                fields[c][tuple(sl)] = 0.0
    return fields


def emission_peak_bin(probe, dt, start):
    """Bin index (and frequency) of the emission peak: |FFT|^2 of the Hann-windowed
    probe record from `start` to its end, argmax on 0.6-0.9 c/a."""
    from paper_0802_3775_amd import analysis as A
    x = np.asarray(probe[start:], dtype=np.float64)
    f, P = A.field_spectrum(x * np.hanning(len(x)), dt)
    band = np.nonzero((f >= 0.6) & (f <= 0.9))[0]
    q = int(band[np.argmax(P[band])])
    return q, float(f[q])
