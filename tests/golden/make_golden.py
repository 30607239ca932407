"""Write the oracle's deviance traces used as targets (D*) by the benchmark.

Calls only the FP64 oracle and the seeded input generators.  Output:
tests/golden/oracle_trace_<name>.json with the full deviance after every
epoch of the seeded schedule, for the workloads:
  c1: Poisson 1000 x 500, d = 5, 200 epochs (and 4 more schedule seeds, to
      measure the seed-to-seed spread of the final deviance);
  c2: NB(alpha=5) 10000 x 2000, d = 10, p = 3, q = 1, 200 epochs;
  c3: NB(alpha=5) 100000 x 5000, d = 20, p = 3, q = 1, 200 epochs (full
      deviance every 10 epochs).
Run: python tests/golden/make_golden.py [c1|c2 ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import gmf_oracle as G  # noqa: E402
from synth import CONFIGS, make_problem  # noqa: E402


def trace(name, epochs, seed_shift=0, eval_every=1):
    pr = make_problem(name)
    cfg = G.Config(family=pr.family, link=pr.link, phi=pr.phi, nb_alpha=pr.nb_alpha,
                   R=pr.R, S=pr.S, seed=pr.sched_seed + seed_shift)
    o = G.OracleGMF(cfg, pr.Y, pr.X, pr.Z, pr.B0, pr.A0, pr.U0, pr.V0)
    devs = [o.full_deviance()]
    evals = [0]
    t0 = time.time()
    for e in range(epochs):
        o.epoch()
        if (e + 1) % eval_every == 0 or e + 1 == epochs:
            devs.append(o.full_deviance())
            evals.append(e + 1)
        if (e + 1) % 10 == 0:
            print(f"{name} seed+{seed_shift} epoch {e + 1} dev {devs[-1]:.6f} "
                  f"({time.time() - t0:.0f}s)", flush=True)
    return dict(workload=name, config=CONFIGS[name], schedule_seed=cfg.seed,
                rate0=cfg.rate0, decay=cfg.decay, tau=cfg.tau, alpha1=cfg.alpha1,
                alpha2=cfg.alpha2, damping=cfg.damping, lam=list(cfg.lam),
                epochs=epochs, eval_epochs=evals, deviance_per_epoch=devs, final=devs[-1])


def main(names):
    for name in names:
        out = trace(name, 200, eval_every=10 if name == "c3" else 1)
        if name == "c1":
            out["seed_spread_finals"] = [trace(name, 200, k)["final"] for k in range(1, 5)]
        path = os.path.join(HERE, f"oracle_trace_{name}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print("wrote", path, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c2"])
