"""Shared set-up for the GPU tests: build the oracle and the HIP path from the
same seeded problem, and the relative error metric used for parity."""
import numpy as np

from oracle import gmf_oracle as G


def rel_err(x, ref):
    """max |x - ref| / max |ref| (norm-wise relative error)."""
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    if ref.size == 0:
        return 0.0
    return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-30))


def oracle_for(pr, **over):
    kw = dict(family=pr.family, link=pr.link, phi=pr.phi, nb_alpha=pr.nb_alpha,
              R=pr.R, S=pr.S, seed=pr.sched_seed)
    kw.update(over)
    cfg = G.Config(**kw)
    return G.OracleGMF(cfg, pr.Y, pr.X, pr.Z, pr.B0, pr.A0, pr.U0, pr.V0, W=pr.W)


def gpu_for(pr, precision="fp32", **over):
    from paper_2412_20509_amd.gmf import GMF, FitConfig
    kw = dict(family=pr.family, link=pr.link, precision=precision, d=pr.d, R=pr.R, S=pr.S,
              phi=pr.phi, nb_alpha=pr.nb_alpha, seed=pr.sched_seed)
    if "lam" in over:
        over["lam"] = tuple(over["lam"])
    kw.update(over)
    fc = FitConfig(**kw)
    X = pr.X if pr.p > 0 else None
    Z = pr.Z if pr.q > 0 else None
    B0 = pr.B0 if pr.p > 0 else None
    A0 = pr.A0 if pr.q > 0 else None
    return GMF(fc, pr.Y, X, Z, B0, A0, pr.U0, pr.V0, W=pr.W)


def compare_state(g, o, tol, what=""):
    """Check every output array of the GPU context against the oracle."""
    B, A, U, V = g.params()
    Gr, Hr, Gc, Hc = g.moments()
    errs = {
        "B": rel_err(B, o.B), "Gamma": rel_err(A, o.A), "U": rel_err(U, o.U),
        "V": rel_err(V, o.V), "Grow": rel_err(Gr, o.Grow), "Hrow": rel_err(Hr, o.Hrow),
        "Gcol": rel_err(Gc, o.Gcol), "Hcol": rel_err(Hc, o.Hcol),
    }
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, f"{what}: relative errors above {tol}: {bad} (all: {errs})"
    return errs
