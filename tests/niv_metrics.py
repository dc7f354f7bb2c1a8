"""Error metrics of the parity tests.

FP32 bar (max relative error 1e-5): the error of an output is measured
relative to its own magnitude, or to the magnitude of the terms summed into
it when cancellation makes the output smaller than its terms.  That term
magnitude is the network evaluated with |W| on |x| along the active ReLU
units of the FP64 forward pass; rounding in any FP32 evaluation is relative
to it (plain sequential FP32 matrix products of the same network reach
2.5e-9 of it, but 1.4e-4 relative to a floor of 1e-3 of the largest output).

FP16/BF16 bar: per-image relative L2 error 2e-3 against the FP64 oracle
evaluated on the same rounded parameters."""
import numpy as np


def term_scale(mats, x0):
    """|W_H| ... |W_0| |x0| along the ReLU units active in the FP64 pass."""
    h = x0.T
    a = np.abs(x0).T
    for Wm in mats[:-1]:
        z = Wm @ h
        act = z > 0
        h = np.where(act, z, 0.0)
        a = (np.abs(Wm) @ a) * act
    return (np.abs(mats[-1]) @ a).T


def max_rel_fp32(E, E_ref, scale):
    return float(np.max(np.abs(E - E_ref) / np.maximum(np.abs(E_ref), np.maximum(scale, 1e-30))))


def max_rel_floored(a, b, frac=1e-3):
    floor = frac * np.abs(b).max()
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), floor)))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def assert_flags(fl, fl_ref, E_ref, near):
    """Flags are integer outputs and must agree exactly, except the
    negative-output bit (16), whose sign test may go either way where an
    output channel lies within `near` of zero (`near` per output, from the
    bar of the precision)."""
    np.testing.assert_array_equal(fl & 0xEF, fl_ref & 0xEF)
    diff = ((fl ^ fl_ref) & 16) != 0
    if diff.any():
        close = (np.abs(E_ref) <= near).any(axis=1)
        bad = np.nonzero(diff & ~close)[0]
        assert bad.size == 0, ("negative-output flag differs away from zero", bad[:10])


def sign_margin(prec, E_ref, scale):
    """How close to zero an output may be for its sign to be undecided:
    1e-5 of the term scale for FP32, 1e-3 of it for FP16/BF16 (the 16-bit
    queries stay within ~6e-6 of the term scale on the room frame, so this
    leaves two orders of magnitude for other models and frames)."""
    if prec == "fp32":
        return 1e-5 * np.maximum(np.abs(E_ref), scale)
    return 1e-3 * np.maximum(np.abs(E_ref), scale)


def relu_margin(mats, x0):
    """Per sample, the smallest |z| / (|W| |h|) over the hidden units, z the
    pre-activation and |W| |h| the magnitude of its terms, in the FP64 pass.
    Where it is below the FP32 rounding of z (~1e-7), an FP32 evaluation may
    take the other ReLU decision; the gradient then gates a different unit.
    Both decisions are correct to the precision, so gradient comparisons
    leave such samples out (on both sides)."""
    h = x0.T
    m = np.full(x0.shape[0], np.inf)
    for Wm in mats[:-1]:
        z = Wm @ h
        sc = np.abs(Wm) @ np.abs(h)
        r = np.abs(z) / np.maximum(sc, 1e-300)
        m = np.minimum(m, r.min(axis=0))
        h = np.maximum(z, 0.0)
    return m
