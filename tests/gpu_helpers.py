"""Helpers shared by the GPU parity tests (operand upload, oracle checks)."""
import numpy as np

from oracle import core


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def fp64_tolerance(c_ref, s_ref, k):
    """Allowed |c_hat - c| for an FP64 dot product of length k: the classic
    gamma_k (|A||B|)_ij bound plus the Dot2 reference's own u|c|."""
    return core.gamma(max(k, 1)) * s_ref + 2 * core.U * np.abs(c_ref)


def check_sampled(A, B, C_hat, rows, cols, k=None):
    """Compare sampled entries of C_hat with the Dot2 oracle; returns max
    scaled error |c_hat - c| / s."""
    c, s = core.sampled(A, B, rows, cols)
    got = C_hat[rows, cols]
    k = A.shape[1] if k is None else k
    tol = fp64_tolerance(c, s, k)
    bad = np.abs(got - c) > tol
    assert not bad.any(), ("%d of %d sampled entries outside the FP64 bound; first at (%d, %d): "
                           "got %r want %r" % (bad.sum(), bad.size, rows[bad][0], cols[bad][0],
                                               got[bad][0], c[bad][0]))
    with np.errstate(divide="ignore", invalid="ignore"):
        sc = np.where(s > 0, np.abs(got - c) / s, 0.0)
    return float(sc.max()) if sc.size else 0.0


def check_freivalds(A, B, C_hat, seeds=(1, 2, 3)):
    from paper_1306_4161_amd import inputs
    for sd in seeds:
        x = inputs.rademacher(B.shape[1], sd)
        r, bd = core.freivalds(A, B, C_hat, x)
        assert np.all(r <= bd), "Freivalds check failed (seed %d): max ratio %g" % (
            sd, float(np.max(r / np.maximum(bd, 1e-300))))
