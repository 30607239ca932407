"""Write the oracle's deviance traces used as targets (D*) by the benchmark.

Calls only the FP64 oracle and the seeded input generators.  Output:
tests/golden/oracle_trace_<name>.json with the full deviance after every
epoch of the seeded schedule, for the workloads:
  c1: Poisson 1000 x 500, d = 5, 200 epochs (and 4 more schedule seeds, to
      measure the seed-to-seed spread of the final deviance);
  c2: NB(alpha=5) 10000 x 2000, d = 10, p = 3, q = 1, 200 epochs;
  c3: NB(alpha=5) 100000 x 5000, d = 20, p = 3, q = 1, 200 epochs (full
      deviance every 10 epochs).
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
