#!/usr/bin/env python
"""Benchmark of block-wise adaptive SGD for GMF on one MI355X.

Headline workload: negative binomial GMF (alpha = 5, log link),
n = 100,000 x m = 5,000, rank d = 20, row covariates X = [1, batch indicator,
N(0,1)] (p = 3), Z = 1 (q = 1), about 85 % zeros, blocks of 10 % of the rows x
20 % of the columns (10000 x 1000, R = 10, S = 5).  Y is 2 GB of int32.

One benchmark "step" is one epoch: R*S = 50 block steps of Algorithm 1 (block
select, eta, inverse link, D1/D2, the four contractions, EMA and step, block
deviance) followed by one evaluation of the full deviance.  Inputs are resident
in HBM before the timed region starts.  --warmup epochs run untimed on a
throwaway context, then exactly --steps epochs are timed.

Printed JSON line:
  value             epochs/s of the headline arm (--headline, default BF16:
                    bfloat16 operands on the matrix cores, float32
                    accumulation, float64 moments and deviance sums), over the
                    --steps timed epochs with the deviance of every epoch
  s_to_1e4          seconds from the first launch until the evaluation of the
                    full deviance that is first within 1e-4 (relative) of D*,
                    the FP64 oracle's deviance after 200 epochs of the same
                    seeded schedule (tests/golden/oracle_trace_c3.json),
                    completed on the device.  Measured by a separate
                    convergence run of --budget epochs (whatever --steps is),
                    the deviance of every epoch evaluated on the device after
                    the epoch's steps, in order on the same stream
  arms              per arm (FP32 plain, BF16, split BF16): epochs/s with and
                    without the per-epoch deviance, s and epochs to 1e-4 of D*,
                    the final distance to D*, the launch statistics
  roofline          the headline arm's step kernel (the launches that run the
                    block-step tiles, level_kernel): algorithmic work per
                    launch (the per-step figure times the steps per launch) /
                    the mean launch time from HIP events stamped by the
                    launches themselves on the library's stream.  The
                    bfloat16 arms are rated on bytes against 8 TB/s HBM: 4 B of
                    y per block entry plus the panel and moment traffic
                    2 (|I| (q+d) + |J| (p+d)) (4 + 2 x 8) B per step; the FP32
                    arm on flops against the 157.3 TFLOP/s float32 peak:
                    2 (3p + 3q + 5d) per block entry.  With the counts held
                    as 16-bit integers (compact_counts) the tiles read 2 B
                    per entry: stored_GBs / stored_frac_hbm rate the launch
                    on those bytes.  traffic = measured HBM
                    bytes per launch (rocprofv3 counters, summary under
                    profiles/), null when the kernel changed since
  from_initialization  the headline arm started from the paper's
                    initialization (Section 4.1, gmf_initialize) instead of the
                    random start: its time, and the seconds (including it) and
                    epochs to 1e-4 of the same D*
  cpu_baseline      the FP64 oracle on the host, a bounded sample of block
                    steps of the same workload, with all threads and with one
  small             the 10000 x 2000 rank-10 workload (FP32 plain path over its
                    200 epochs and the bfloat16 arms), against its own D*
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


PREC_CODE = {"fp32": 0, "bf16": 1, "bf16x3": 2}


def step_kernel_name(pr, precision, compact):
    """Template name of the step kernel that runs a workload: level_kernel<
    precision, family, panel stride, block deviance, wavefronts per tile,
    16-bit counts>."""
    fam = {"poisson": 0, "negbin": 1, "gaussian": 2}[pr.family]
    k = pr.p + pr.q + pr.d
    # automatic panel stride: k rounded up to 16 (FP32, or k <= 16), else to 32
    stride = (k + 15) // 16 * 16 if (precision == "fp32" or k <= 16) else (k + 31) // 32 * 32
    cy = "true" if compact and precision != "fp32" else "false"
    return f"level_kernel<{PREC_CODE[precision]}, {fam}, {stride}, true, 4, {cy}>"


def recorded_traffic(pr, precision, compact):
    """HBM bytes per launch of a workload's step kernel from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None when the summary has no
    line for the kernel or the kernel sources (step.hip, family.hpp, mfma.hpp)
    changed since those counters were taken."""
    import glob
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("step.hip", "family.hpp", "mfma.hpp"):
        with open(os.path.join(ROOT, "paper_2412_20509_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    src = h.hexdigest()[:16]
    want = step_kernel_name(pr, precision, compact)
    shape = f"{pr.n}x{pr.m}"
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_*.md"))):
        for m in re.finditer(r"traffic_bytes_per_launch: (\d+) source: ([0-9a-f]+) "
                             r"kernel: (level_kernel<[^>]*>) workload: (\S+)",
                             open(path).read()):
            if m.group(3) == want and m.group(4) == shape and m.group(2) == src:
                return float(m.group(1))
    return None


FP32_PEAK_TFS = 157.3


def step_work(pr, bf16):
    """Algorithmic work of one block step (the per-entry figures times the
    block's entries): bytes = 4 B of y per entry plus the panel and moment
    traffic 2 (|I| (q+d) + |J| (p+d)) (4 + 2 s) with s = 8 B (float64 moments)
    on the bfloat16 paths and 4 B on the FP32 path; flops = 2 (3p + 3q + 5d)
    per entry (eta, the two U-side and the two V-side contractions).
    bytes_stored: the same with the 2 B per entry the step tiles read when
    the counts are held as 16-bit integers."""
    ns, ms = pr.n / pr.R, pr.m / pr.S
    s_mom = 8.0 if bf16 else 4.0
    panels = 2.0 * (ns * (pr.q + pr.d) + ms * (pr.p + pr.d)) * (4.0 + 2.0 * s_mom)
    return dict(bytes=4.0 * ns * ms + panels, bytes_stored16=2.0 * ns * ms + panels,
                flops=2.0 * (3 * pr.p + 3 * pr.q + 5 * pr.d) * ns * ms)


def run_arm(pr, precision, epochs, warmup, budget, dstar, torch, polish=0):
    """One arm: `warmup` untimed epochs on a throwaway context; exactly `epochs`
    timed epochs, each followed by the full deviance on the device (gmf_run);
    the same epochs without the deviance; a separate convergence run of
    `budget` epochs with the deviance of every epoch, for the seconds and
    epochs to 1e-4 of D*; HIP-event launch statistics over 2 more epochs.
    polish > 0: the last `polish` epochs of the convergence run switch from
    BF16 to FP32 steps (gmf_set_precision) on the same iterate."""
    per_epoch = pr.R * pr.S
    g = make_gmf(pr, precision)
    for _ in range(warmup):
        g.step(per_epoch)
        g.deviance()
    g.close()
    del g
    torch.cuda.synchronize()

    # the timed region: `epochs` epochs, the full deviance of every epoch
    g = make_gmf(pr, precision)
    compact = g.compact_counts
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.run(epochs, eval_every=1)
    wall = time.perf_counter() - t0
    # the same epochs without the deviance evaluations, then the launch
    # statistics of 2 more epochs from HIP events on the library's stream
    g.close()
    g = make_gmf(pr, precision)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g.run(epochs, trace=False)
    wall_steps = time.perf_counter() - t1
    g.set_timing(True)
    for _ in range(2):
        g.step(per_epoch)
    (tile_ms, tile_launches), (upd_ms, upd_launches) = g.get_timing_by_kind()
    launch_ms, launches, nsteps = g.get_timing()
    g.set_timing(False)
    g.close()
    del g

    # convergence: `budget` epochs from the start, deviance every epoch
    g = make_gmf(pr, precision)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if polish > 0:
        devs, ms = g.run(budget - polish, eval_every=1)
        t_mid = time.perf_counter() - t0
        g.set_precision("fp32")
        d2, m2 = g.run(polish, eval_every=1)
        devs, ms = devs + d2, ms + [1e3 * t_mid + x for x in m2]
    else:
        devs, ms = g.run(budget, eval_every=1)
    conv_wall = time.perf_counter() - t0
    t_hit = e_hit = None
    rel_at_200 = None
    if dstar is not None:
        e, t = first_hit(devs, ms, dstar)
        if e is not None:
            t_hit, e_hit = t / 1e3, e + 1
        if len(devs) >= 200:
            rel_at_200 = abs(devs[199] - dstar) / dstar
    t_pp = time.perf_counter()
    g.params(postprocess=1)
    t_pp = time.perf_counter() - t_pp
    final = devs[-1]
    g.close()
    return dict(epochs=epochs, wall_s=wall, epochs_per_s=epochs / wall,
                ms_per_epoch=1e3 * wall / epochs,
                epochs_per_s_without_deviance=epochs / wall_steps,
                budget_epochs=budget, budget_wall_s=conv_wall,
                final_deviance=final,
                rel_to_oracle_final=(abs(final - dstar) / dstar) if dstar else None,
                rel_to_oracle_at_epoch_200=rel_at_200,
                deviance_at_epoch_200=devs[199] if len(devs) >= 200 else None,
                deviance_every_10_epochs=devs[9::10],
                s_to_1e4=t_hit, epochs_to_1e4=e_hit,
                launch_ms_total=launch_ms, launches=int(launches), timed_steps=nsteps,
                tile_launch_ms_total=tile_ms, tile_launches=int(tile_launches),
                update_launch_ms_total=upd_ms, update_launches=int(upd_launches),
                postprocess_s=t_pp, compact_counts=compact)


def run_init_arm(pr, precision, budget, dstar, torch, power_iters=2, oversample=6):
    """The paper's initialization (Section 4.1, least-squares form, gmf_initialize)
    in place of the random start, then `budget` epochs with the deviance of
    every epoch: the initialization's time and the seconds (including it) and
    epochs to 1e-4 of D* (the random-start oracle's 200-epoch deviance)."""
    import numpy as np
    Om = np.random.default_rng(6000 + pr.n % 1000).normal(size=(pr.m, pr.d + oversample))
    Omd = torch.as_tensor(Om.astype(np.float32), device="cuda:0")
    g = make_gmf(pr, precision)             # warm-up of the initialization kernels
    g.initialize(Omd, power_iters=power_iters)
    g.close()
    g = make_gmf(pr, precision)
    d0, _ = g.deviance()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.initialize(Omd, power_iters=power_iters)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    d_init, _ = g.deviance()
    t1 = time.perf_counter()
    devs, ms = g.run(budget, eval_every=1)
    wall = time.perf_counter() - t1
    g.close()
    out = dict(init_s=t_init, deviance_random_start=d0, deviance_after_init=d_init,
               power_iters=power_iters, k=pr.d + oversample, budget_epochs=budget,
               budget_wall_s=wall, final_deviance=devs[-1], s_to_1e4=None, epochs_to_1e4=None)
    if dstar is not None:
        e, t = first_hit(devs, ms, dstar)
        if e is not None:
            out["epochs_to_1e4"] = e + 1
            out["s_to_1e4"] = t_init + t / 1e3
        out["final_rel_below_dstar"] = (dstar - devs[-1]) / dstar
    return out


def roofline_of(pr, arm, precision):
    """Roofline object of an arm's step kernel, the dominant kernel: the
    launches that run the block-step tiles (level_kernel).  Every block entry
    of the timed steps is processed in those launches, so their algorithmic
    work per launch is the per-step figure times the steps per tile launch;
    the launch durations are HIP events stamped by the launches themselves on
    the library's stream (see the module docstring).  `step_kernels_*` rate
    the same work over the tile and the update launches together."""
    bf16 = precision != "fp32"
    w = step_work(pr, bf16)
    steps = arm["timed_steps"]
    n_tile = max(arm["tile_launches"], 1)
    t_tile = arm["tile_launch_ms_total"] * 1e-3
    t_all = arm["launch_ms_total"] * 1e-3
    per_launch_bytes = w["bytes"] * steps / n_tile
    per_launch_flops = w["flops"] * steps / n_tile
    mean_s = t_tile / n_tile
    if bf16:
        achieved = per_launch_bytes / mean_s / 1e9
        out = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                   frac=achieved / HBM_PEAK_GBS,
                   step_kernels_GBs=steps * w["bytes"] / t_all / 1e9)
    else:
        achieved = per_launch_flops / mean_s / 1e12
        out = dict(bound="mfma", achieved=achieved, peak=FP32_PEAK_TFS, unit="TFLOP/s",
                   frac=achieved / FP32_PEAK_TFS,
                   step_kernels_TFs=steps * w["flops"] / t_all / 1e12)
    compact = bool(arm.get("compact_counts")) and precision != "fp32"   # FP32 tiles read float32
    traffic = recorded_traffic(pr, precision, compact)
    name = step_kernel_name(pr, precision, compact)
    # launches of at most one tile per compute unit run the 8-wavefront variant
    stride = int(name.split(", ")[2])
    nw8 = (precision == "fp32" and stride in (16, 32)) or (precision != "fp32" and stride == 32)
    variants = [name] + ([name.replace(", 4, true>", ", 8, false>").replace(", 4, false>", ", 8, false>")]
                         if nw8 else [])
    out.update(traffic=traffic, kernel=name, kernel_variants=variants,
               bytes_per_step=w["bytes"], flops_per_step=w["flops"],
               algorithmic_bytes_per_launch=per_launch_bytes,
               algorithmic_flops_per_launch=per_launch_flops,
               counts_bytes_per_entry=2 if compact else 4,
               steps_per_launch=steps / n_tile, mean_launch_us=1e6 * mean_s,
               launches=int(n_tile), update_launches=arm["update_launches"],
               mean_update_launch_us=1e6 * arm["update_launch_ms_total"] * 1e-3 /
               max(arm["update_launches"], 1))
    if compact:
        # the bytes the tiles have to move with 16-bit counts, against HBM
        out["stored_GBs"] = w["bytes_stored16"] * steps / n_tile / mean_s / 1e9
        out["stored_frac_hbm"] = out["stored_GBs"] / HBM_PEAK_GBS
    if traffic is not None:
        # the same launch time against the bytes the HBM counters measured
        out["measured_GBs"] = traffic / mean_s / 1e9
        out["measured_frac_hbm"] = out["measured_GBs"] / HBM_PEAK_GBS
        out["traffic_over_algorithmic"] = traffic / per_launch_bytes
    return out


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
    # the FP64 oracle's D* on its seeded 1 % subset of the new rows (rows are
    # independent: projecting the subset alone equals the full projection
    # restricted to it): each arm's distance to it and epochs to 1e-4 of it
    oracle_subset = None
    gold = os.path.join(ROOT, "tests", "golden", "oracle_warm_subset_c5.json")
    if os.path.exists(gold) and n_new == json.load(open(gold))["n_new"]:
        gs = json.load(open(gold))
        idx = torch.as_tensor(np.asarray(gs["rows"], np.int64), device="cuda:0")
        Ys, Xs = Yd[idx].contiguous(), Xd[idx].contiguous()
        cs = enc.forward(Ys, bf16=True)
        oracle_subset = dict(rows=gs["subset_rows"], dstar=gs["dstar"],
                             oracle_last_rel_change=gs["last_rel_change"])
        for name, prec, cand in (("cold", "fp32", None), ("warm", "fp32", cs),
                                 ("warm_bf16x3", "bf16x3", cs), ("warm_bf16", "bf16", cs)):
            g.set_precision(prec)
            _, _, trs, mss, _ = g.project_warm(Ys, Xs, cand, max_epochs, frozen=1, trace=True)
            g.set_precision("fp32")
            es, _ = first_hit(trs, mss, gs["dstar"])
            oracle_subset[name] = dict(final_rel_to_oracle_dstar=abs(trs[-1] - gs["dstar"]) /
                                       gs["dstar"], epochs_to_1e4_of_oracle_dstar=es)
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
        oracle_subset=oracle_subset,
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


def gen_batched(nfits, scale):
    """The seeded problems of the batched-fits workload (host arrays)."""
    from synth import gen_nb
    log(f"batched fits: generating {nfits} problems (scale {scale})")
    return [gen_nb(n=sp["n"], m=sp["m"], d=sp["d"], R=10, S=5, seed=sp["seed"],
                   family=sp["family"], chunked=True) for sp in batch_specs(nfits, scale)]


def run_batched(nfits, scale, epochs, torch, tile_rows=384, precision="fp32", solo=True,
                problems=None, modes=((1, "graph"), (2, "leveled")), solo_tile_rows=128):
    """Many uneven fits: fit-by-fit epochs (each context stepped on its own,
    `solo_tile_rows`-row tiles) against batched epochs (gmf_batch_*: the fixed
    launch sequence as a recorded graph, and level placement; `tile_rows`-row
    tiles).  Fits are grouped into batches by panel stride (p + q + d <= 32 ->
    32, else 48, 64 for the bfloat16 precisions); the batches run on their own
    streams, side by side.  tile_rows 0: the library's rule, -1: the
    autotuner's table (the first fit of each shape class tuned).  In a batch
    the other fits supply the parallelism, so deeper tiles than a single fit
    wants pay (fewer tiles, each pipelining more row groups)."""
    from paper_2412_20509_amd.gmf import Batch, FitConfig, GMF, tune, tune_lookup
    if problems is None:
        problems = gen_batched(nfits, scale)
    tuned = {}
    entries = sum(pr.n * pr.m for pr in problems)

    def contexts(rows):
        out = []
        for pr in problems:
            stride = 32 if pr.k <= 32 else (48 if precision == "fp32" else 64)
            fc = FitConfig(family=pr.family, d=pr.d, R=pr.R, S=pr.S, nb_alpha=pr.nb_alpha,
                           seed=pr.sched_seed, panel_stride=stride, skip_block_deviance=1,
                           tile_rows=max(rows, 0), precision=precision)
            if rows < 0:
                fc.tile_rows = 0
                cfg = fc.to_c(pr.n, pr.m, pr.p, pr.q)
                if tune_lookup(cfg) == 0:
                    best, _ = tune(fc, pr.Y, pr.X, pr.Z, pr.B0, pr.A0, pr.U0, pr.V0,
                                   candidates=(64, 128, 256, 512), steps=20)
                    tuned[best] = tuned.get(best, 0) + 1
            out.append(GMF(fc, pr.Y, pr.X, pr.Z, pr.B0, pr.A0, pr.U0, pr.V0, device="cuda:0"))
        torch.cuda.synchronize()
        return out

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def close(fits):
        for g in fits:
            g.close()
        torch.cuda.empty_cache()

    t_solo = None
    if solo:
        fits = contexts(solo_tile_rows)
        timed(lambda: [g.step(g.cfg.R * g.cfg.S) for g in fits])      # warm-up epoch
        t_solo = timed(lambda: [g.step(g.cfg.R * g.cfg.S) for _ in range(epochs) for g in fits])
        close(fits)
    fits = contexts(tile_rows)
    groups = {}
    for g in fits:
        groups.setdefault(g.cfg.panel_stride, []).append(g)
    res = {}
    for mode, name in modes:
        batches = [Batch(gs, table_epochs=max(epochs, 1), mode=mode) for gs in groups.values()]
        for b in batches:
            b.run(1, trace=False)                                   # warm-up epoch
        t = timed(lambda: [b.run(epochs, trace=False) for b in batches])
        res[name] = t
        for b in batches:
            b.close()
    close(fits)
    del fits
    out = dict(
        workload=(f"{nfits} fits: family coin Poisson/NB, n ~ U{{2000..50000}} x {scale}, "
                  f"m ~ U{{1000..5000}} x {scale}, d ~ U{{5..30}}, p = 3, q = 1, blocks 10 % x 20 %"),
        entries=entries, epochs=epochs, groups={int(k): len(v) for k, v in groups.items()},
        tile_rows=tile_rows if tile_rows >= 0 else "autotuned", tuned_classes=tuned,
        separate_tile_rows=solo_tile_rows if solo else None, precision=precision,
        separate_epochs_per_s=None if t_solo is None else epochs / t_solo)
    for name, t in res.items():
        out[f"batched_{name}_epochs_per_s"] = epochs / t
        out[f"batched_{name}_count_GBs"] = 4.0 * entries * epochs / t / 1e9
    if "leveled" in res:
        out["batched_leveled_hbm_frac_counts"] = out["batched_leveled_count_GBs"] / HBM_PEAK_GBS
        if t_solo is not None:
            out["speedup_vs_separate"] = t_solo / res["leveled"]
    return out


def cpu_info():
    """Host CPU model and logical CPU count (nproc) of the machine this runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return model, nproc


def cpu_baseline(pr, steps=8, steps_1t=3, dev_rows=2000):
    """The FP64 oracle (numpy) on a bounded sample of the workload: `steps`
    block steps of the seeded schedule and the full deviance over `dev_rows`
    rows (scaled to all n rows), with the BLAS pool at its default size and
    again with one thread; an epoch is R*S steps plus one full deviance."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import gmf_oracle as G
    cfg = G.Config(family=pr.family, link=pr.link, phi=pr.phi, nb_alpha=pr.nb_alpha,
                   R=pr.R, S=pr.S, seed=pr.sched_seed)
    o = G.OracleGMF(cfg, pr.Y, pr.X, pr.Z, pr.B0, pr.A0, pr.U0, pr.V0)
    rows = np.arange(min(dev_rows, pr.n))

    def sample(k):
        t0 = time.perf_counter()
        o.steps(k)
        t_step = (time.perf_counter() - t0) / k
        t0 = time.perf_counter()
        mu = G.inverse_link(cfg.link, o.eta_full(rows), cfg.eps, cfg.eta_max)
        float(G.unit_deviance(cfg.family, o.Y[rows], mu, cfg.nb_alpha).sum())
        t_dev = (time.perf_counter() - t0) * pr.n / len(rows)
        return t_step, t_dev

    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    t_step, t_dev = sample(steps)
    with threadpool_limits(limits=1):
        t_step1, t_dev1 = sample(steps_1t)
    per_epoch = pr.R * pr.S
    ep = per_epoch * t_step + t_dev
    ep1 = per_epoch * t_step1 + t_dev1
    model, nproc = cpu_info()
    return dict(value=1.0 / ep, unit="epochs/s", cores=threads, kind="oracle",
                sample=(f"{steps} block steps of {pr.n // pr.R}x{pr.m // pr.S} (seeded schedule, "
                        f"from the start) and the full deviance over {len(rows)} of {pr.n} "
                        f"rows of the same {pr.n}x{pr.m} NB workload, FP64 numpy; epoch = "
                        f"{per_epoch} steps + 1 full deviance"),
                single_thread_value=1.0 / ep1, cpu_model=model, nproc=nproc,
                seconds_per_step=t_step, seconds_per_step_1_thread=t_step1,
                full_deviance_s=t_dev, full_deviance_s_1_thread=t_dev1)


DTYPE = {"fp32": "f32", "bf16": "bf16", "bf16x3": "bf16x3"}


def run_arms(pr, arms_arg, epochs, warmup, budget, dstar, torch, tag):
    arms = {}
    for arm in arms_arg.split(","):
        prec, polish = arm, 0
        if arm == "bf16+fp32":             # BF16, then FP32 for the last quarter
            prec, polish = "bf16", budget // 4
        log(f"{tag} arm {arm}: {warmup} warm-up + {epochs} timed epochs, "
            f"{budget}-epoch convergence run")
        arms[arm] = run_arm(pr, prec, epochs, warmup, budget, dstar, torch, polish=polish)
        arms[arm]["roofline"] = roofline_of(pr, arms[arm], prec)
        log(f"{tag} arm {arm}: {arms[arm]['epochs_per_s']:.1f} epochs/s, "
            f"s to 1e-4: {arms[arm]['s_to_1e4']} ({arms[arm]['epochs_to_1e4']} epochs), "
            f"roofline frac {arms[arm]['roofline']['frac']:.3f}")
    return arms


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed epochs per arm")
    ap.add_argument("--warmup", type=int, default=2, help="untimed warm-up epochs per arm")
    ap.add_argument("--budget", type=int, default=400,
                    help="epochs of each arm's convergence run (s to 1e-4 of D*)")
    ap.add_argument("--arms", default="fp32,bf16,bf16x3",
                    help="fp32, bf16, bf16x3 (split bfloat16), bf16+fp32 (BF16 steps, "
                         "FP32 for the last quarter of the convergence run)")
    ap.add_argument("--headline", default="bf16", help="arm whose epochs/s is `value`")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-init", action="store_true",
                    help="skip the arm that starts from the paper's initialization")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the 10000x2000 rank-10 section")
    ap.add_argument("--small-epochs", type=int, default=200)
    ap.add_argument("--small-budget", type=int, default=300)
    ap.add_argument("--no-warm", action="store_true", help="skip the warm-start section")
    ap.add_argument("--warm-rows", type=int, default=1_000_000)
    ap.add_argument("--warm-epochs", type=int, default=60,
                    help="projection epochs per arm (the reference runs 3x as many)")
    ap.add_argument("--encoder-epochs", type=int, default=40)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-fits section")
    ap.add_argument("--batch-fits", type=int, default=64)
    ap.add_argument("--batch-scale", type=float, default=1.0,
                    help="factor on n and m of every batched fit")
    ap.add_argument("--batch-epochs", type=int, default=5)
    ap.add_argument("--batch-tile-rows", type=int, default=384,
                    help="rows per tile of the batched fits (0: the library's rule, "
                         "-1: the autotuner's table, tuned on the first fit of each shape class)")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the batched-fits section and print its result")
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
    if args.only_batched:      # the batched-fits section alone (for profiling)
        probs = gen_batched(args.batch_fits, args.batch_scale)
        out = run_batched(args.batch_fits, args.batch_scale, args.batch_epochs, torch,
                          tile_rows=args.batch_tile_rows, problems=probs)
        out["bf16"] = run_batched(args.batch_fits, args.batch_scale, args.batch_epochs, torch,
                                  tile_rows=args.batch_tile_rows, precision="bf16", solo=False,
                                  problems=probs, modes=((2, "leveled"),))
        print(json.dumps(out))
        return
    log("generating the 100000x5000 NB workload (rank 20)")
    pr = make_problem("c3")
    target = load_target("c3")
    dstar = target["final"] if target and target.get("epochs_done") == target.get("epochs") \
        else None
    arms = run_arms(pr, args.arms, args.steps, args.warmup, args.budget, dstar, torch, "c3")
    head = arms.get(args.headline) or next(iter(arms.values()))
    head_name = args.headline if args.headline in arms else next(iter(arms))
    init_arm = None
    if not args.no_init:
        log(f"c3 arm {head_name} from the paper's initialization: {args.budget} epochs")
        init_arm = run_init_arm(pr, head_name.split("+")[0], args.budget, dstar, torch)
        log(f"initialization {init_arm['init_s'] * 1e3:.1f} ms; s to 1e-4: {init_arm['s_to_1e4']} "
            f"({init_arm['epochs_to_1e4']} epochs)")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on the host")
        cpu = cpu_baseline(pr)
    workload = ("NB GMF 100000x5000, d=20, p=3, q=1, alpha=5, blocks 10000x1000 (R=10, S=5); "
                "step = 1 epoch (50 block steps + full deviance)")
    config = dict(workload=workload, n=pr.n, m=pr.m, d=pr.d, p=pr.p, q=pr.q, R=pr.R, S=pr.S,
                  zero_fraction=float((pr.Y == 0).mean()), arm=head_name,
                  comparison_arm="fp32")
    del pr

    small = None
    if not args.no_small:
        log("generating the 10000x2000 NB workload")
        pr2 = make_problem("c2")
        t2 = load_target("c2")
        small = dict(workload="NB GMF 10000x2000, d=10, p=3, q=1, alpha=5, blocks 1000x400",
                     oracle_final_deviance=t2["final"] if t2 else None,
                     arms=run_arms(pr2, "fp32,bf16,bf16x3", args.small_epochs, args.warmup,
                                   args.small_budget, t2["final"] if t2 else None, torch, "c2"))
        pr2_keep = pr2
    warm = None
    if not args.no_warm:
        pr2w = pr2_keep if small is not None else make_problem("c2")
        warm = run_warm_start(pr2w, args.warm_rows, args.warm_epochs, args.encoder_epochs, torch)
        log(f"warm start: cold {warm['cold']['epochs_to_1e4']} epochs, "
            f"warm {warm['warm']['epochs_to_1e4']} epochs, "
            f"warm bf16x3 {warm['warm_bf16x3']['epochs_to_1e4']} epochs, "
            f"warm bf16 {warm['warm_bf16']['epochs_to_1e4']} epochs, "
            f"{warm['warm']['fallback_rows']} fallback rows")
    batched = None
    if not args.no_batched:
        probs = gen_batched(args.batch_fits, args.batch_scale)
        batched = run_batched(args.batch_fits, args.batch_scale, args.batch_epochs, torch,
                              tile_rows=args.batch_tile_rows, problems=probs)
        batched["bf16"] = run_batched(args.batch_fits, args.batch_scale, args.batch_epochs, torch,
                                      tile_rows=args.batch_tile_rows, precision="bf16",
                                      solo=False, problems=probs, modes=((2, "leveled"),))
        del probs
        log(f"batched fits: {batched['batched_leveled_epochs_per_s']:.1f} epochs/s batched "
            f"(level placement), {batched['batched_graph_epochs_per_s']:.1f} (fixed graph), "
            f"{batched['separate_epochs_per_s']:.1f} separately")

    out = dict(
        metric=METRIC, value=head["epochs_per_s"], unit="epochs/s", n_gpus=1,
        steps=args.steps, warmup=args.warmup, ms_per_step=head["ms_per_epoch"],
        higher_is_better=True, scaling="weak", vs_baseline=None, dtype=DTYPE[head_name.split("+")[0]],
        data="synthetic", config=config,
        s_to_1e4=head["s_to_1e4"], epochs_to_1e4=head["epochs_to_1e4"],
        s_to_1e4_by_arm={k: v["s_to_1e4"] for k, v in arms.items()},
        epochs_per_s_by_arm={k: v["epochs_per_s"] for k, v in arms.items()},
        oracle_final_deviance=dstar, roofline=head["roofline"], cpu_baseline=cpu,
        arms=arms, from_initialization=init_arm, small=small, warm_start=warm,
        batched=batched,
    )
    print(json.dumps(out))


if __name__ == "__main__":
    main()
