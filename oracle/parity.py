"""Parity criterion of the GPU path against the oracle (test infrastructure
only; used by the test-suite and the smoke check).

Every floating-point comparison measures, per state s, the max-normalised
error against the extended-precision evaluation of the same definition
(oracle.extended):

    e_s(x) = max_i |x_si - ext_si| / max_i |ext_si|

and requires

    e_s(GPU) <= max(tol, factor * e_s(FP64 oracle))

with tol = 1e-12 and factor = 2 unless a test states otherwise. The first term
is the plain 1e-12 relative bar. The second applies only where no FP64
evaluation can reach that bar: where the result is a small difference of large
terms, the FP64 oracle's own error against the extended evaluation measures
that conditioning directly (for the smooth Mach-0.1 vortex on fine meshes the
density residual is pure truncation error, about 1e-7 of the terms it is
summed from), and the GPU must then be no less accurate than plain FP64
evaluation, within the factor.

"The FP64 oracle's own error" is the larger of the errors of the FP64
evaluations passed in (the PyTorch oracle and the plain-FP64 coding of the
extended module, where both are available). On non-degenerate states two such
codings agree within a factor of about 1.3; on states whose exact value is
zero up to round-off (a velocity component that vanishes at every node) they
differ by up to an order of magnitude, and the larger one is the honest
estimate of FP64 noise there.
"""
import numpy as np


def state_errors(x, ext):
    """e_s(x) for arrays of shape (S, ...) (numpy, torch or long double)."""
    ext = np.asarray(ext, dtype=np.longdouble)
    x = np.asarray(_np(x)).astype(np.longdouble)
    S = ext.shape[0]
    d = np.abs(x - ext).reshape(S, -1).max(1)
    m = np.abs(ext).reshape(S, -1).max(1)
    m = np.where(m > 0, m, np.longdouble(1e-300))
    return (d / m).astype(np.float64)


def _np(x):
    if hasattr(x, "detach"):
        return x.detach().cpu().double().numpy()
    return x


def check(got, ext, ref64, tol=1e-12, factor=2.0):
    """Return (ok, e_gpu, e_64, bound) per state for the criterion above;
    ref64 is one FP64 evaluation or a list of them."""
    e_gpu = state_errors(got, ext)
    refs = ref64 if isinstance(ref64, (list, tuple)) else [ref64]
    e_64 = np.max(np.stack([state_errors(r, ext) for r in refs]), axis=0)
    bound = np.maximum(tol, factor * e_64)
    return bool(np.all(e_gpu <= bound)), e_gpu, e_64, bound


def describe(e_gpu, e_64, bound):
    return ("GPU " + np.array2string(e_gpu, precision=2) + " | FP64 oracle "
            + np.array2string(e_64, precision=2) + " | bound " + np.array2string(bound, precision=2))
