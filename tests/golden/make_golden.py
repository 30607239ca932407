"""Write the oracle's deviance traces used as targets (D*) by the benchmark.

Calls only the FP64 oracle and the seeded input generators.  Output:
tests/golden/oracle_trace_<name>.json with the full deviance after every
epoch of the seeded schedule, for the workloads:
  c1: Poisson 1000 x 500, d = 5, 200 epochs (and 4 more schedule seeds, to
      measure the seed-to-seed spread of the final deviance);
  c2: NB(alpha=5) 10000 x 2000, d = 10, p = 3, q = 1, 200 epochs;
  c3: NB(alpha=5) 100000 x 5000, d = 20, p = 3, q = 1, 200 epochs (full
      deviance every 10 epochs);
  c5: the learned warm start's D* on a seeded 1 % subset of its 1,000,000
      new rows (oracle fit, Algorithm 2, oracle projection of the subset;
      tests/golden/oracle_warm_subset_c5.json).
Run: python tests/golden/make_golden.py [c1|c2|c3 ...] [--checkpoint DIR]

With --checkpoint DIR the oracle's whole state (parameters, moments, step
counter, trace so far) is saved to DIR every 10 epochs and a run resumes from
it; a partial trace (epochs_done < epochs) is written next to the final file
as oracle_trace_<name>.partial.json while the run is in progress.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import gmf_oracle as G  # noqa: E402
from synth import CONFIGS, make_problem  # noqa: E402

_STATE = ("B", "A", "U", "V", "Grow", "Hrow", "Gcol", "Hcol")


def _save_state(path, o, devs, evals):
    tmp = path + ".tmp.npz"
    np.savez(tmp, t=o.t, devs=np.asarray(devs), evals=np.asarray(evals),
             **{k: getattr(o, k) for k in _STATE})
    os.replace(tmp, path)


def _load_state(path, o):
    with np.load(path, allow_pickle=False) as z:
        for k in _STATE:
            getattr(o, k)[...] = z[k]
        o.t = int(z["t"])
        return list(z["devs"]), [int(e) for e in z["evals"]]


def _record(name, cfg, epochs, evals, devs):
    return dict(workload=name, config=CONFIGS[name], schedule_seed=cfg.seed,
                rate0=cfg.rate0, decay=cfg.decay, tau=cfg.tau, alpha1=cfg.alpha1,
                alpha2=cfg.alpha2, damping=cfg.damping, lam=list(cfg.lam),
                epochs=epochs, epochs_done=evals[-1], eval_epochs=evals,
                deviance_per_epoch=devs, final=devs[-1])


def trace(name, epochs, seed_shift=0, eval_every=1, ckpt_dir=None):
    pr = make_problem(name)
    cfg = G.Config(family=pr.family, link=pr.link, phi=pr.phi, nb_alpha=pr.nb_alpha,
                   R=pr.R, S=pr.S, seed=pr.sched_seed + seed_shift)
    o = G.OracleGMF(cfg, pr.Y, pr.X, pr.Z, pr.B0, pr.A0, pr.U0, pr.V0)
    del pr
    steps_per_epoch = cfg.R * cfg.S
    ckpt = None
    if ckpt_dir is not None:
        os.makedirs(ckpt_dir, exist_ok=True)
        ckpt = os.path.join(ckpt_dir, f"oracle_state_{name}_s{seed_shift}.npz")
    if ckpt is not None and os.path.exists(ckpt):
        devs, evals = _load_state(ckpt, o)
        print(f"{name}: resumed at step {o.t}", flush=True)
    else:
        devs, evals = [o.full_deviance()], [0]
    partial = os.path.join(HERE, f"oracle_trace_{name}.partial.json")
    t0 = time.time()
    for e in range(o.t // steps_per_epoch, epochs):
        o.epoch()
        if (e + 1) % eval_every == 0 or e + 1 == epochs:
            devs.append(o.full_deviance())
            evals.append(e + 1)
        if (e + 1) % 10 == 0:
            print(f"{name} seed+{seed_shift} epoch {e + 1} dev {devs[-1]:.6f} "
                  f"({time.time() - t0:.0f}s)", flush=True)
            if ckpt is not None:
                _save_state(ckpt, o, devs, evals)
                if seed_shift == 0:
                    with open(partial, "w") as f:
                        json.dump(_record(name, cfg, epochs, evals, devs), f, indent=1)
    return _record(name, cfg, epochs, evals, devs)


def warm_subset(n_new=1_000_000, frac=0.01, epochs=180, subset_seed=5006):
    """D* of the learned warm-start workload on a seeded 1 % subset of its new
    rows: the oracle's 200-epoch fit of the 10000 x 2000 NB workload, its
    Algorithm 2 column side, and the oracle's projection of the subset rows
    from the cold start (row intercept, U = 0) run for `epochs` epochs (rows
    are independent, so the subset's projection is the full projection
    restricted to it).  Records the subset's row indices, the deviance trace
    of the subset every 10 epochs and its last relative change."""
    from synth import gen_nb_rows
    pr = make_problem("c2")
    cfg = G.Config(family=pr.family, link=pr.link, phi=pr.phi, nb_alpha=pr.nb_alpha,
                   R=pr.R, S=pr.S, seed=pr.sched_seed)
    o = G.OracleGMF(cfg, pr.Y, pr.X, pr.Z, pr.B0, pr.A0, pr.U0, pr.V0)
    t0 = time.time()
    for e in range(200):
        o.epoch()
        if (e + 1) % 50 == 0:
            print(f"c5: oracle fit epoch {e + 1} ({time.time() - t0:.0f}s)", flush=True)
    B, _, _, V = G.postprocess_A_B1(pr.X, pr.Z, o.B, o.A, o.U, o.V)
    Ynew, Xnew, _, _ = gen_nb_rows(pr, n_new, seed=5005)
    rows = np.sort(np.random.default_rng(subset_seed).choice(n_new, int(frac * n_new),
                                                             replace=False))
    Ys = np.asarray(Ynew[rows])
    Xs = np.asarray(Xnew[rows], np.float64)
    del Ynew, Xnew
    cols = G.partition(G.permutation(cfg.seed, G.STREAM_COLS, pr.m), pr.S)
    A0 = G.row_intercept_start(cfg, Ys, Xs, B, pr.q)
    U0 = np.zeros((len(rows), pr.d))
    rec = []
    G.project_rows(cfg, Ys, Xs, pr.Z, B, V, A0, U0, epochs, cols, record=rec)
    # the subset's deviance at the start and after every 10th epoch (S steps each)
    trace = [float(G.row_deviance(cfg, Ys, Xs, pr.Z, B, A0, U0, V).sum())]
    for e in range(10, epochs + 1, 10):
        A, U = rec[e * pr.S - 1]
        trace.append(float(G.row_deviance(cfg, Ys, Xs, pr.Z, B, A, U, V).sum()))
    return dict(workload="learned warm start: new NB rows of the 10000x2000 workload's column side",
                n_new=n_new, subset_rows=int(len(rows)), subset_seed=subset_seed,
                rows=[int(r) for r in rows], epochs=epochs, deviance_every_10_epochs=trace,
                last_rel_change=abs(trace[-1] - trace[-2]) / trace[-1], dstar=trace[-1],
                fit_epochs=200, fit_final_deviance=o.full_deviance())


def main(argv):
    ckpt_dir = None
    names = []
    it = iter(argv)
    for a in it:
        if a == "--checkpoint":
            ckpt_dir = next(it)
        else:
            names.append(a)
    for name in names or ["c1", "c2"]:
        if name == "c5":
            out = warm_subset()
            path = os.path.join(HERE, "oracle_warm_subset_c5.json")
            with open(path, "w") as f:
                json.dump(out, f)
            print("wrote", path, flush=True)
            continue
        out = trace(name, 200, eval_every=10 if name == "c3" else 1, ckpt_dir=ckpt_dir)
        if name == "c1":
            out["seed_spread_finals"] = [trace(name, 200, k)["final"] for k in range(1, 5)]
        path = os.path.join(HERE, f"oracle_trace_{name}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        partial = os.path.join(HERE, f"oracle_trace_{name}.partial.json")
        if os.path.exists(partial):
            os.remove(partial)
        print("wrote", path, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
