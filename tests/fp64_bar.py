"""The FP64 parity bar, applied event by event.

The GPU's FP64 result must be within 1e-12 (relative) of the exact |M|^2 of
the event.  The FP64 oracle is that value only to its own rounding, which
ill-conditioned events (nearly collinear massless legs: strong cancellations
between diagrams and small invariants) amplify to 1e-11 and beyond.  So every
event on which the GPU and the FP64 oracle differ by more than 1e-13 is
re-evaluated with the long-double oracle (64-bit mantissa, colour algebra in
long double as well), and there the GPU must be within 1e-12 of it: on that
same event, with no allowance taken from the FP64 oracle's own error.
"""
import numpy as np

FLAG = 1e-13
BAR = 1e-12


def check_fp64(gpu, ref, long_double, label="", flag=FLAG, median=1e-14):
    """gpu, ref: GPU and FP64-oracle |M|^2 of the same events;
    long_double(idx) returns the long-double oracle's values of events idx.
    flag=0 sends every event to long double; median (None: no check) bounds
    the median GPU/FP64-oracle difference, a sanity check on well-conditioned
    inputs.  Returns (flagged count, worst GPU error against long double)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    assert np.isfinite(gpu).all() and (gpu > 0).all(), label
    rel = np.abs(gpu / ref - 1.0)
    if median is not None:
        assert np.median(rel) <= median, (label, np.median(rel))
    flagged = np.nonzero(rel > flag)[0] if flag > 0 else np.arange(rel.size)
    worst = 0.0
    if flagged.size:
        ld = np.asarray(long_double(flagged))
        e_gpu = np.abs(gpu[flagged] / ld - 1.0)
        e_ora = np.abs(ref[flagged] / ld - 1.0)
        worst = float(e_gpu.max())
        print(f"  {label} {flagged.size} of {rel.size} events above {flag:g} against the FP64 oracle; "
              f"against long double: GPU worst {worst:.3e}, FP64 oracle worst {e_ora.max():.3e}", flush=True)
        bad = flagged[e_gpu > BAR]
        assert bad.size == 0, (label, bad.tolist()[:10], e_gpu[e_gpu > BAR].tolist()[:10])
    else:
        print(f"  {label} max rel {rel.max():.3e} median {np.median(rel):.3e} (none above {flag:g})", flush=True)
    return flagged.size, worst
