#!/usr/bin/env python
"""Benchmark of block-wise adaptive SGD for GMF on one MI355X.

Workload (the headline configuration): negative binomial GMF (alpha = 5, log
link), n = 10,000 x m = 2,000, rank d = 10, row covariates X = [1, batch
indicator, N(0,1)] (p = 3), Z = 1 (q = 1), about 85 % zeros, blocks of 10 % of
the rows x 20 % of the columns (R = 10, S = 5), plain FP32 path.

One benchmark "step" is one epoch: R*S = 50 block steps of Algorithm 1 (block
select, eta, inverse link, D1/D2, the four contractions, EMA and step, block
deviance) followed by one evaluation of the full deviance.  Inputs are resident
in HBM before the timed region starts.

Printed JSON line:
  value             epochs/s of the FP32 arm (whole job, one GPU)
  s_to_1e-4         seconds from the first launch until the evaluation of the
                    full deviance that is first within 1e-4 (relative) of D*,
                    the FP64 oracle's deviance after 200 epochs of the same
                    seeded schedule (tests/golden), completed on the device;
                    the deviance of every epoch is evaluated on the device
                    after the epoch's steps, in order on the same stream
  roofline          dominant kernel (the fused tile kernel): algorithmic
                    bytes per launch / mean launch time from HIP events stamped
                    by the launches themselves on the library's stream, against
                    the 8 TB/s HBM peak; traffic = measured HBM bytes per launch
                    (rocprofv3 counters, summary under profiles/)
  cpu_baseline      the FP64 oracle on the host, bounded sample
  arms              the same measurements for each arm: FP32, BF16, split BF16
                    (bf16x3), optionally BF16 steps finished by FP32 steps over
                    the last quarter of the epochs (bf16+fp32)
  large             the 100000 x 5000 rank-20 workload (steps only), per precision
  batched           64 uneven fits advanced together (gmf_batch_*) against the
                    same fits stepped one by one
  warm_start        learned warm start of 1,000,000 new rows: epochs and
                    seconds to 1e-4 of the converged projection deviance for a
                    cold start and for the encoder's bfloat16 predictions, with
                    FP32, split-BF16 and BF16 projection steps
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GMF SGD epochs/s + s to 1e-4 rel deviance; BF16/warm vs FP32 plain"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def load_target(name):
    path = os.path.join(ROOT, "tests", "golden", f"oracle_trace_{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def make_gmf(pr, precision):
    from paper_2412_20509_amd.gmf import GMF, FitConfig
    fc = FitConfig(family=pr.family, link=pr.link, precision=precision, d=pr.d, R=pr.R,
                   S=pr.S, phi=pr.phi, nb_alpha=pr.nb_alpha, seed=pr.sched_seed)
    return GMF(fc, pr.Y, pr.X, pr.Z, pr.B0, pr.A0, pr.U0, pr.V0, device="cuda:0")


def recorded_traffic():
    """HBM bytes per launch of the headline step kernel from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None when the kernel sources
    (step.hip, family.hpp, mfma.hpp) changed since those counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "hbm_traffic_level_kernel_nb10000x2000_nb100000x5000.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"traffic_bytes_per_launch: (\d+) source: ([0-9a-f]+)", open(path).read())
    if not m:
        return None
    h = hashlib.sha256()
    for f in ("step.hip", "family.hpp", "mfma.hpp"):
        with open(os.path.join(ROOT, "paper_2412_20509_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return float(m.group(1)) if h.hexdigest()[:16] == m.group(2) else None


def tile_bytes_per_launch(pr):
    """Algorithmic bytes of one tile-kernel launch: the block's counts (4 B each)
    plus one read of the block's two panels (p+q+d floats per row/column)."""
    ns, ms = pr.n / pr.R, pr.m / pr.S
    return 4.0 * ns * ms + 4.0 * (ns + ms) * pr.k


def run_arm(pr, precision, epochs, warmup, dstar, torch, polish=0):
    """Timed epochs of one arm; polish > 0: the last `polish` epochs switch
    from BF16 to FP32 steps (gmf_set_precision) on the same iterate."""
    per_epoch = pr.R * pr.S
    # warm-up on a throwaway context (kernel loading, caches)
    g = make_gmf(pr, precision)
    for _ in range(warmup):
        g.step(per_epoch)
        g.deviance()
    g.close()
    del g
    torch.cuda.synchronize()

    g = make_gmf(pr, precision)
    torch.cuda.synchronize()
    # the timed region: `epochs` epochs, the full deviance of every epoch
    # evaluated after the epoch's steps on the same stream (gmf_run)
    t0 = time.perf_counter()
    if polish > 0:
        devs, ms = g.run(epochs - polish, eval_every=1)
        t_mid = time.perf_counter() - t0
        g.set_precision("fp32")
        d2, m2 = g.run(polish, eval_every=1)
        devs, ms = devs + d2, ms + [1e3 * t_mid + x for x in m2]
    else:
        devs, ms = g.run(epochs, eval_every=1)
    wall = time.perf_counter() - t0
    t_hit = e_hit = None
    if dstar is not None:
        for e, (dv, t) in enumerate(zip(devs, ms)):
            if abs(dv - dstar) <= 1e-4 * dstar:
                t_hit, e_hit = t / 1e3, e + 1
                break
    # the same epochs without the deviance evaluations (steps only)
    g2 = make_gmf(pr, precision)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if polish > 0:
        g2.run(epochs - polish, trace=False)
        g2.set_precision("fp32")
        g2.run(polish, trace=False)
    else:
        g2.run(epochs, trace=False)
    wall_steps = time.perf_counter() - t1
    g2.close()
    del g2

    # HIP events around every step launch on the library's stream (2 more epochs)
    g.set_timing(True)
    for _ in range(2):
        g.step(per_epoch)
        g.deviance()
    launch_ms, launches, nsteps = g.get_timing()
    g.set_timing(False)
    t_pp = time.perf_counter()
    g.params(postprocess=1)
    t_pp = time.perf_counter() - t_pp
    final = devs[-1]
    g.close()
    return dict(epochs=epochs, wall_s=wall, epochs_per_s=epochs / wall,
                ms_per_epoch=1e3 * wall / epochs,
                epochs_per_s_without_deviance=epochs / wall_steps, final_deviance=final,
                rel_to_oracle=(abs(final - dstar) / dstar) if dstar else None,
                s_to_1e4=t_hit, epochs_to_1e4=e_hit,
                launch_ms_total=launch_ms, launches=int(launches), timed_steps=nsteps,
                postprocess_s=t_pp)


def run_throughput(pr, precision, epochs, torch):
    """Steps-only throughput of a large workload: epochs/s, launch roofline and
    the time of one full-deviance evaluation."""
    per_epoch = pr.R * pr.S
    g = make_gmf(pr, precision)
    g.step(per_epoch)                  # warm-up epoch
    torch.cuda.synchronize()
    g.set_timing(True)
    t0 = time.perf_counter()
    g.step(epochs * per_epoch)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms, launches, nsteps = g.get_timing()
    g.set_timing(False)
    t1 = time.perf_counter()
    dev, _ = g.deviance()
    t_dev = time.perf_counter() - t1
    g.close()
    bytes_step = tile_bytes_per_launch(pr)
    achieved = nsteps * bytes_step / (launch_ms * 1e-3) / 1e9
    return dict(epochs=epochs, epochs_per_s=epochs / wall, ms_per_epoch=1e3 * wall / epochs,
                launches=int(launches), steps=nsteps, launch_ms_total=launch_ms,
                bytes_per_step=bytes_step, achieved_GBs=achieved, hbm_frac=achieved / HBM_PEAK_GBS,
                deviance_eval_s=t_dev, deviance=dev)


def first_hit(trace, ms, target, rel=1e-4):
    """(epoch, wall ms) of the first deviance within rel of target, else (None, None)."""
    for e, (dv, t) in enumerate(zip(trace, ms)):
        if abs(dv - target) <= rel * target:
            return e, t
    return None, None


def run_warm_start(pr, n_new, max_epochs, enc_epochs, torch):
    """Learned warm start of new rows: fit the workload, train the encoder on
    (log1p counts, projected scores) of its rows (90/10 split), then project
    n_new fresh rows from the same generator cold (U0 = 0) and warm (U0 =
    encoder output in bfloat16, per-row fallback to 0), all with the row
    intercept start, the warm start with FP32, split-BF16 and BF16 projection
    steps, and time each to 1e-4 of the converged projection deviance."""
    import numpy as np
    from paper_2412_20509_amd.gmf import Encoder
    from synth import gen_nb_rows, mlp_init
    per_epoch = pr.R * pr.S
    g = make_gmf(pr, "fp32")
    g.step(200 * per_epoch)
    torch.cuda.synchronize()
    n_tr = int(0.9 * pr.n)
    Ytr = torch.as_tensor(pr.Y, device="cuda:0")
    # encoder targets: the optimum of each fitted row's own projection problem on
    # the frozen column side (the scores a projection converges to), so that the
    # encoder learns the map the warm start is meant to shortcut
    _, Uft, _, _, _ = g.project_warm(Ytr, pr.X, None, 3 * max_epochs, frozen=1)
    enc = Encoder(pr.m, pr.d, mlp_init(pr.m, 256, pr.d), hidden=256, batch=256, lr=1e-3)
    t0 = time.perf_counter()
    losses = enc.train(Ytr[:n_tr], Uft[:n_tr], enc_epochs)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    val = enc.forward(Ytr[n_tr:], bf16=True)
    val_mse = float(((val - Uft[n_tr:]) ** 2).mean())
    val_var = float(((Uft[n_tr:] - Uft[n_tr:].mean(0)) ** 2).mean())
    del Ytr, Uft
    log(f"warm start: generating {n_new} new rows")
    Ynew, Xnew, _, _ = gen_nb_rows(pr, n_new, seed=5005)
    Yd = torch.as_tensor(Ynew, device="cuda:0")
    Xd = torch.as_tensor(np.asarray(Xnew, np.float32), device="cuda:0")
    del Ynew
    # converged reference: a cold run to a relative change below 1e-9 (or the cap)
    log("warm start: converged reference (cold)")
    _, _, ref, _, _ = g.project_warm(Yd, Xd, None, 3 * max_epochs, frozen=1, trace=True)
    ref_change = abs(ref[-1] - ref[-2]) / ref[-1]
    dstar = ref[-1]
    log("warm start: cold arm")
    _, _, trc, msc, _ = g.project_warm(Yd, Xd, None, max_epochs, frozen=1, trace=True)
    log("warm start: warm arm")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cand = enc.forward(Yd, bf16=True)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    _, _, trw, msw, fb = g.project_warm(Yd, Xd, cand, max_epochs, frozen=1, trace=True)
    # the same warm start with split-bfloat16 and bfloat16 projection steps on
    # the same fitted context (panel stride 16: 16x16x16 bfloat16 products)
    bfa = {}
    for prec in ("bf16x3", "bf16"):
        log(f"warm start: warm arm, {prec} steps")
        g.set_precision(prec)
        _, _, trx, msx, fbx = g.project_warm(Yd, Xd, cand, max_epochs, frozen=1, trace=True)
        g.set_precision("fp32")
        ex, tx = first_hit(trx, msx, dstar)
        bfa[prec] = dict(epochs_to_1e4=ex, s_to_1e4=None if tx is None else tx / 1e3 + t_inf,
                         deviance_start=trx[0], fallback_rows=fbx,
                         final_rel_to_reference=abs(trx[-1] - dstar) / dstar,
                         ms_per_epoch=(msx[-1] - msx[0]) / max_epochs)
    ec, tc = first_hit(trc, msc, dstar)
    ew, tw = first_hit(trw, msw, dstar)
    enc.close()
    g.close()
    return dict(
        workload=(f"{n_new} new NB rows x {pr.m} (same column side, fresh rows), projected "
                  f"on the frozen Algorithm 2 column side of the {pr.n}x{pr.m} fit"),
        encoder=dict(train_rows=n_tr, val_rows=pr.n - n_tr, epochs=enc_epochs,
                     train_loss_first=losses[0], train_loss_last=losses[-1],
                     val_mse_bf16=val_mse, val_target_var=val_var, train_s=t_train,
                     infer_s=t_inf, infer_rows_per_s=n_new / t_inf),
        reference=dict(epochs=3 * max_epochs, deviance=dstar, last_rel_change=ref_change),
        cold=dict(epochs_to_1e4=ec, s_to_1e4=None if tc is None else tc / 1e3,
                  deviance_start=trc[0], ms_per_epoch=(msc[-1] - msc[0]) / max_epochs),
        warm=dict(epochs_to_1e4=ew,
                  s_to_1e4=None if tw is None else tw / 1e3 + t_inf,
                  deviance_start=trw[0], fallback_rows=fb,
                  ms_per_epoch=(msw[-1] - msw[0]) / max_epochs),
        warm_bf16x3=bfa["bf16x3"],
        warm_bf16=bfa["bf16"],
    )


def batch_specs(nfits, scale, seed=1004):
    """Shapes of the batched-fits workload: per fit a seeded coin for the family
    (Poisson / NB), n ~ U{2000..50000}, m ~ U{1000..5000}, d ~ U{5..30}, with
    n and m multiplied by `scale`; blocks of 10 % x 20 % (R = 10, S = 5)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    for i in range(nfits):
        fam = "negbin" if rng.random() < 0.5 else "poisson"
        n = int(rng.integers(2000, 50001) * scale)
        m = int(rng.integers(1000, 5001) * scale)
        d = int(rng.integers(5, 31))
        out.append(dict(family=fam, n=n, m=m, d=d, seed=seed * 100 + i))
    return out


def run_batched(nfits, scale, epochs, torch):
    """Many uneven fits: fit-by-fit epochs (each context stepped on its own)
    against batched epochs (gmf_batch_*, with and without the recorded graph).
    Fits are grouped into batches by panel stride (p + q + d <= 32 -> 32,
    else 48); every fit uses 128-row tiles."""
    from paper_2412_20509_amd.gmf import Batch, FitConfig, GMF
    from synth import gen_nb
    specs = batch_specs(nfits, scale)
    log(f"batched fits: generating {nfits} problems (scale {scale})")
    fits, entries = [], 0
    for sp in specs:
        pr = gen_nb(n=sp["n"], m=sp["m"], d=sp["d"], R=10, S=5, seed=sp["seed"],
                    family=sp["family"], chunked=True)
        stride = 32 if pr.k <= 32 else 48
        # 128-row tiles: in a batch the other fits supply the parallelism, and
        # deeper tiles pipeline their row groups (61 vs 51 epochs/s at 32 rows)
        fc = FitConfig(family=pr.family, d=pr.d, R=pr.R, S=pr.S, nb_alpha=pr.nb_alpha,
                       seed=pr.sched_seed, panel_stride=stride, skip_block_deviance=1,
                       tile_rows=128)
        fits.append(GMF(fc, pr.Y, pr.X, pr.Z, pr.B0, pr.A0, pr.U0, pr.V0, device="cuda:0"))
        entries += pr.n * pr.m
        del pr
    torch.cuda.synchronize()
    groups = {}
    for g in fits:
        groups.setdefault(g.cfg.panel_stride, []).append(g)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def solo():
        for _ in range(epochs):
            for g in fits:
                g.step(g.cfg.R * g.cfg.S)

    timed(lambda: [g.step(g.cfg.R * g.cfg.S) for g in fits])      # warm-up epoch
    t_solo = timed(solo)
    res = {}
    for use_graph in (False, True):
        batches = [Batch(gs, table_epochs=max(epochs, 1), use_graph=use_graph)
                   for gs in groups.values()]
        for b in batches:
            b.run(1, trace=False)                                   # warm-up epoch
        t = timed(lambda: [b.run(epochs, trace=False) for b in batches])
        res["graph" if use_graph else "direct"] = t
        for b in batches:
            b.close()
    for g in fits:
        g.close()
    return dict(
        workload=(f"{nfits} fits: family coin Poisson/NB, n ~ U{{2000..50000}} x {scale}, "
                  f"m ~ U{{1000..5000}} x {scale}, d ~ U{{5..30}}, p = 3, q = 1, blocks 10 % x 20 %"),
        entries=entries, epochs=epochs, groups={int(k): len(v) for k, v in groups.items()},
        separate_epochs_per_s=epochs / t_solo,
        batched_epochs_per_s=epochs / res["direct"],
        batched_graph_epochs_per_s=epochs / res["graph"],
        batched_graph_entries_per_s=entries * epochs / res["graph"],
        speedup_vs_separate=t_solo / res["graph"],
    )


def cpu_baseline(pr, epochs=3):
    from threadpoolctl import threadpool_info
    from oracle import gmf_oracle as G
    cfg = G.Config(family=pr.family, link=pr.link, phi=pr.phi, nb_alpha=pr.nb_alpha,
                   R=pr.R, S=pr.S, seed=pr.sched_seed)
    o = G.OracleGMF(cfg, pr.Y, pr.X, pr.Z, pr.B0, pr.A0, pr.U0, pr.V0)
    t0 = time.perf_counter()
    for _ in range(epochs):
        o.epoch()
        o.full_deviance()
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return dict(value=epochs / dt, unit="epochs/s", cores=threads, kind="oracle",
                sample=f"{epochs} epochs ({epochs * pr.R * pr.S} block steps of "
                       f"{pr.n // pr.R}x{pr.m // pr.S}, each epoch followed by one full "
                       f"deviance) of the same {pr.n}x{pr.m} NB workload, FP64 numpy",
                seconds=dt)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed epochs")
    ap.add_argument("--warmup", type=int, default=3, help="untimed warm-up epochs")
    ap.add_argument("--arms", default="fp32,bf16,bf16x3",
                    help="fp32, bf16, bf16x3 (split bfloat16), bf16+fp32 (BF16 steps, "
                         "FP32 for the last quarter)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 100000x5000 rank-20 throughput section")
    ap.add_argument("--large-epochs", type=int, default=5)
    ap.add_argument("--no-warm", action="store_true", help="skip the warm-start section")
    ap.add_argument("--warm-rows", type=int, default=1_000_000)
    ap.add_argument("--warm-epochs", type=int, default=60,
                    help="projection epochs per arm (the reference runs 3x as many)")
    ap.add_argument("--encoder-epochs", type=int, default=40)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-fits section")
    ap.add_argument("--batch-fits", type=int, default=64)
    ap.add_argument("--batch-scale", type=float, default=0.5,
                    help="factor on n and m of every batched fit")
    ap.add_argument("--batch-epochs", type=int, default=5)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 3 device-to-device copies of MIB MiB (a plain copy "
                         "kernel of known size, to scale HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {nbytes} bytes 3 times")
        return
    from synth import make_problem
    from paper_2412_20509_amd import gmf as _gmf  # noqa: F401  (fails if not built)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log("generating the 10000x2000 NB workload")
    pr = make_problem("c2")
    target = load_target("c2")
    dstar = target["final"] if target else None

    arms = {}
    for arm in args.arms.split(","):
        prec, polish = arm, 0
        if arm == "bf16+fp32":             # BF16, then FP32 for the last quarter
            prec, polish = "bf16", args.steps // 4
        log(f"arm {arm}: {args.warmup} warm-up + {args.steps} timed epochs")
        arms[arm] = run_arm(pr, prec, args.steps, args.warmup, dstar, torch, polish=polish)
        log(f"arm {arm}: {arms[arm]['epochs_per_s']:.1f} epochs/s, "
            f"s to 1e-4: {arms[arm]['s_to_1e4']}")

    main_arm = arms.get("fp32") or next(iter(arms.values()))
    bytes_step = tile_bytes_per_launch(pr)
    bytes_launch = bytes_step * main_arm["timed_steps"] / max(main_arm["launches"], 1)
    mean_launch_s = main_arm["launch_ms_total"] * 1e-3 / max(main_arm["launches"], 1)
    achieved = bytes_launch / mean_launch_s / 1e9
    roof = dict(bound="hbm", kernel="level_kernel<0, 1, 16, true, 4>", achieved=achieved,
                peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                traffic=recorded_traffic(), bytes_per_launch=bytes_launch,
                mean_launch_us=1e6 * mean_launch_s, steps_per_launch=main_arm["timed_steps"] /
                max(main_arm["launches"], 1))
    large = None
    if not args.no_large:
        log("generating the 100000x5000 NB workload (rank 20)")
        pr3 = make_problem("c3")
        large = {}
        for prec in ("bf16x3", "bf16", "fp32"):
            log(f"large workload, arm {prec}: 1 warm-up + {args.large_epochs} timed epochs")
            large[prec] = run_throughput(pr3, prec, args.large_epochs, torch)
            log(f"large {prec}: {large[prec]['epochs_per_s']:.1f} epochs/s, "
                f"{large[prec]['achieved_GBs']:.0f} GB/s")
        large["workload"] = ("NB GMF 100000x5000, d=20, p=3, q=1, alpha=5, blocks 10000x1000 "
                             "(R=10, S=5); steps only, one full deviance timed separately")
        del pr3
    warm = None
    if not args.no_warm:
        warm = run_warm_start(pr, args.warm_rows, args.warm_epochs, args.encoder_epochs, torch)
        log(f"warm start: cold {warm['cold']['epochs_to_1e4']} epochs, "
            f"warm {warm['warm']['epochs_to_1e4']} epochs, "
            f"warm bf16x3 {warm['warm_bf16x3']['epochs_to_1e4']} epochs, "
            f"warm bf16 {warm['warm_bf16']['epochs_to_1e4']} epochs, "
            f"{warm['warm']['fallback_rows']} fallback rows")
    batched = None
    if not args.no_batched:
        batched = run_batched(args.batch_fits, args.batch_scale, args.batch_epochs, torch)
        log(f"batched fits: {batched['batched_graph_epochs_per_s']:.1f} epochs/s batched "
            f"(graph), {batched['separate_epochs_per_s']:.1f} separately")
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on the host")
        cpu = cpu_baseline(pr)

    out = dict(
        metric=METRIC, value=main_arm["epochs_per_s"], unit="epochs/s", n_gpus=1,
        steps=args.steps, warmup=args.warmup, ms_per_step=main_arm["ms_per_epoch"],
        higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
        data="synthetic",
        config=dict(workload="NB GMF 10000x2000, d=10, p=3, q=1, alpha=5, blocks "
                              "1000x400 (R=10, S=5), FP32 plain path, step = 1 epoch "
                              "(50 block steps + full deviance)",
                    n=pr.n, m=pr.m, d=pr.d, p=pr.p, q=pr.q, R=pr.R, S=pr.S,
                    zero_fraction=float((pr.Y == 0).mean())),
        s_to_1e4=main_arm["s_to_1e4"], epochs_to_1e4=main_arm["epochs_to_1e4"],
        oracle_final_deviance=dstar, roofline=roof, cpu_baseline=cpu, large=large,
        warm_start=warm, batched=batched,
        arms={k: {kk: vv for kk, vv in v.items()} for k, v in arms.items()},
    )
    print(json.dumps(out))


if __name__ == "__main__":
    main()
