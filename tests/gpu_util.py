"""Helpers shared by the GPU parity tests (HIP path through the C ABI vs oracle)."""
import numpy as np

from oracle import oracle as O


def canon(x, z, c):
    return O.canonical(x, z, c)


def assert_same_terms(got, ref, what=""):
    """Keys bit-exact; coefficients equal as IEEE values (+0 == -0)."""
    gx, gz, gc = canon(*got)
    rx, rz, rc = canon(*ref)
    assert gx.shape == rx.shape, f"{what}: {gx.shape[0]} terms vs oracle {rx.shape[0]}"
    assert np.array_equal(gx, rx) and np.array_equal(gz, rz), f"{what}: keys differ"
    bad = np.flatnonzero(gc != rc)
    assert bad.size == 0, (f"{what}: {bad.size} coefficients differ, first {bad[:5]}: "
                           f"{gc[bad[:5]]} vs {rc[bad[:5]]}")


def describe(step, what, **kw):
    """Print (and flush) what a GPU step is about to run, so a crash names it."""
    extra = " ".join(f"{k}={v}" for k, v in kw.items())
    print(f"[gpu] {what} step={step} {extra}", flush=True)
