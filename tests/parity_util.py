"""Element-by-element comparison of GPU and oracle fields (test helper)."""
import numpy as np


def assert_fields_close(Ug, Uo, tol=1e-12, what=""):
    """Per field v: max |Ug - Uo| <= tol * max |Uo| and sum |Ug - Uo| <= tol * sum |Uo|.
    A field that nearly vanishes (a momentum at rest) is measured on the scale of
    the density and the energy (the first and last fields), 1e-3 of the larger."""
    Ug, Uo = np.asarray(Ug), np.asarray(Uo)
    scale = np.abs(Uo).reshape(Uo.shape[0], -1).max(axis=1)
    floor = max(scale[0], scale[-1])
    for v in range(Uo.shape[0]):
        d = np.abs(Ug[v] - Uo[v])
        s = max(scale[v], 1e-3 * floor)
        l1 = d.sum() / max(np.abs(Uo[v]).sum(), 1e-3 * floor * d.size)
        assert d.max() <= tol * s, f"{what} field {v}: max |dU| {d.max():.3e} > {tol * s:.3e}"
        assert l1 <= tol, f"{what} field {v}: relative L1 {l1:.3e} > {tol:.1e}"
