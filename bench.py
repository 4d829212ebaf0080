#!/usr/bin/env python3
"""Benchmark of the NEP energy/force/virial MD path on one MI355X.

Workload (one "step" = one full pass of the hot path): velocity-Verlet MD of
the 216,000-bead CG water-like box (60^3 jittered simple-cubic lattice at
33.4 beads/nm^3, Maxwell 300 K), NEP with radial/angular cutoffs 0.8/0.5 nm,
Chebyshev basis 8, n_max 8/6, l_max 4, 30 tanh neurons, random N(0, 0.1^2)
weights; dt = 2 fs, 18 amu; neighbour lists rebuilt every 10 steps on a
0.1 nm skin, and earlier once the two largest displacements since the last
build add up to 0.99 skin (no pair can be missing before) and a pair test then
finds a pair inside a cutoff that was outside the list cutoff at the build
(--plain-skin-test: rebuilt at the first condition alone); beads put back into
cell order every 100 steps.  Each step: half-kick + drift, [wrap +
rebuild], fused descriptor/network/angular-force kernel, gather kernel
(forces + second half-kick + energy sums), FP64 energy reduction.

Two more legs follow (each skippable): the batched fitness form (64
candidates x 2000 structures, persistent launch against the plain
one-structure-per-call loop) and the served form (Poisson trace of MD
requests through the continuous-batching server against a plain FIFO loop).

The timed window is the central K steps of the workload's 1000-step
trajectory from the lattice (the steps before it run untimed), so it sees the
trajectory's typical state: random weights heat the system from 300 K to
about 1350 K, and rebuilds grow more frequent as it heats.  The whole
1000-step trajectory is also timed on its own (`config.full_run`).  Every
step evaluates energies, forces and the per-bead and total virial.

Prints ONE JSON line.  `value` is bead-steps/s with every input resident in
HBM.  The roofline entry prices the dominant kernel's algorithmic FP32 work,
timed with HIP events on its own stream inside the timed region.  The CPU
baseline is the FP64 oracle (the correctness reference, not a tuned CPU code)
on full force evaluations of the same state, on every host core and on one.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NEP force-eval bead-steps/s at 1 GPU; batched/served vs plain; p50/p99 ms"
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector, published
PEAK_HBM_GBS = 8000.0


def algorithmic_flops(nR: np.ndarray, nA: np.ndarray, H: int, T: int):
    """Per-kernel split of the fixed accounting convention (FMA = 2 flops):
         radial pair   2 nR KR + 11 KR + 60, angular pair 4 nA KA + 6 nA L + 14 L + 9 KA + 60,
         per bead      4 H Ndes + 6 H + 4 nA L + 2 nR KR T.
    The fused kernel owns the descriptor sums (2 nR KR + 4 KR + 20 per radial pair),
    every angular and per-bead term; the gather kernel the radial derivatives,
    force and virial (7 KR + 40 per radial pair)."""
    n_R, K_R, n_A, K_A, L, N_des = 9, 9, 7, 9, 24, 37
    rad_main = 2 * n_R * K_R + 4 * K_R + 20
    rad_gather = 7 * K_R + 40
    ang = 4 * n_A * K_A + 6 * n_A * L + 14 * L + 9 * K_A + 60
    bead = 4 * H * N_des + 6 * H + 4 * n_A * L + 2 * n_R * K_R * T
    main = float(nR.sum()) * rad_main + float(nA.sum()) * ang + nR.size * bead
    gather = float(nR.sum()) * rad_gather
    return main, gather


def pair_counts(rep, spec):
    """Neighbours within r_c (not r_c + skin) per bead, from the device lists."""
    from paper_2603_01234_amd.engine import decode_row
    nbr, cnt = rep.neighbor_rows()
    pos = rep.positions(internal=True).astype(np.float64)
    box = np.asarray(rep.box, np.float64)
    n = rep.n
    nR = np.zeros(n, np.int64)
    nA = np.zeros(n, np.int64)
    rcR = float(spec.rc_R.max())
    rcA = float(spec.rc_A.max())
    chunk = 16
    for p0 in range(0, nbr.shape[0], chunk):
        rows = nbr[p0:p0 + chunk]                       # (c, n)
        slot = np.arange(p0, p0 + rows.shape[0])[:, None]
        valid = slot < cnt[0][None, :]
        j, nx, ny, nz = decode_row(rows)
        j = np.where(valid, j, np.arange(n)[None, :])
        d = np.stack([pos[j, 0] + nx * box[0], pos[j, 1] + ny * box[1], pos[j, 2] + nz * box[2]], -1)
        d -= pos[None, :, :]
        r = np.sqrt((d * d).sum(-1))
        nR += (valid & (r < rcR)).sum(0)
        nA += (valid & (slot < cnt[1][None, :]) & (r < rcA)).sum(0)
    return nR, nA


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in ("efv.hip", "efv_device.h", "nep_internal.h"):
        with open(os.path.join(ROOT, "paper_2603_01234_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(n_launch_units: int):
    """HBM bytes per launch of the fused kernel from the committed counter summary,
    or None when the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "efv_main_config1_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        c = json.load(f)
    if c.get("kernel_source_sha256_16") != kernel_hash():
        return None
    return c.get("hbm_bytes_per_launch")


def cpu_baseline(spec, params, system, pos, min_seconds=10.0, single_core_seconds=8.0):
    """The FP64 oracle timed on the host: full force evaluations of the timed
    window's 216,000-bead state on every core of the process, and (the same
    model and density) of a 4,096-bead box on one core."""
    import oracle
    import workloads as W
    p64 = params.astype(np.float32).astype(np.float64)
    box = system.box.astype(np.float32).astype(np.float64)
    cores = oracle.max_threads()
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.efv(spec, p64, pos, system.types, box, system.pbc, n_threads=cores)
        reps += 1
        el = time.perf_counter() - t0
        if el >= min_seconds or reps >= 3:
            break
    small = W.water_box(np.random.SeedSequence(4096), 16, temperature=300.0)
    sp = small.pos_f32().astype(np.float64)
    sb = small.box.astype(np.float32).astype(np.float64)
    t1 = time.perf_counter()
    reps1 = 0
    while True:
        oracle.efv(spec, p64, sp, small.types, sb, small.pbc, n_threads=1)
        reps1 += 1
        el1 = time.perf_counter() - t1
        if el1 >= single_core_seconds:
            break
    oracle.efv(spec, p64, sp, small.types, sb, small.pbc, n_threads=cores)   # back to every core
    return {"value": system.n * reps / el, "unit": "bead-steps/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{reps} full FP64 force evaluation(s) of the 216,000-bead state at the start of the timed "
                      f"window ({el:.1f} s wall, {cores} threads); the MD update itself is negligible",
            "single_core": {"value": small.n * reps1 / el1, "unit": "bead-steps/s", "cores": 1,
                            "sample": f"{reps1} full FP64 force evaluations of a 4,096-bead box of the same "
                                      f"density and model on one thread ({el1:.1f} s wall)"}}


def ensembles_leg(rep, dt, masses, every, steps=100, sort_every=100):
    """The ensemble forms of the MD step on the 216,000-bead state the timed
    window left: NVE for reference, Bussi NVT at 300 K, NPT as calls of 10
    steps (Berendsen barostat at 0.1 GPa with a Berendsen thermostat), and
    HNEMD (F_e = 0.1/nm along z, Berendsen thermostat).  Wall clock over
    `steps` steps each, with the per-bead and total virial every step."""
    import torch
    import oracle
    n = rep.n
    out = {"workload": f"config1 state, {n} beads, {steps} steps per form", "steps": steps}
    rng = np.random.default_rng(2603)
    noise = torch.from_numpy(np.stack([rng.normal(size=steps), rng.chisquare(3 * n - 4, size=steps)], axis=1)).cuda()
    Jt = torch.zeros((steps, 3), dtype=torch.float64, device="cuda")
    Ek = torch.zeros(steps, dtype=torch.float64, device="cuda")
    forms = {
        "nve": None,
        "nvt_bussi": dict(thermostat=2, T_target=300.0, tau_T=100.0, noise=noise),
        "hnemd_berendsen": dict(thermostat=1, T_target=300.0, tau_T=100.0, Fe=(0.0, 0.0, 0.1)),
    }
    for name, ens in forms.items():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep.md(steps, dt, masses, rebuild_every=every, sort_every=sort_every, ensemble=ens,
               E_kin=Ek, J_trace=Jt if name.startswith("hnemd") else None)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[name] = {"ms_per_step": round(el * 1e3 / steps, 4), "bead_steps_per_s": round(n * steps / el, 1),
                     "T_end_K": round(2 * float(Ek[-1]) / ((3 * n - 3) * oracle.KB_EV), 1)}
        if name.startswith("hnemd"):
            out[name]["J_mean_eV_nm_per_fs"] = [round(float(x), 6) for x in Jt.mean(0).cpu().numpy()]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    boxes, P = rep.npt(steps // 10, 10, dt, masses, P_target=(0.1 * 6.241509,) * 3, tau_P=1000.0, beta=0.05,
                       thermostat=1, T_target=300.0, tau_T=100.0, rebuild_every=every)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["npt_berendsen"] = {"ms_per_step": round(el * 1e3 / steps, 4), "bead_steps_per_s": round(n * steps / el, 1),
                            "calls": steps // 10, "P_last_GPa": [round(float(x) / 6.241509, 4) for x in P[-1]],
                            "box_last_nm": [round(float(x), 4) for x in boxes[-1]]}
    out["note"] = ("ensemble steps add four small kernels to the NVE step (sums, drive-free half-kick and commit, "
                   "thermostat factor, velocity scale); NPT is a sequence of 10-step calls, each synchronising once")
    return out


def snes_leg(generations: int = 5):
    """The training loop (Sec. II.A): SNES with 64 candidates on the 1000
    water-like structures of the fitness workload, every step on the device
    (sample, load the candidates, one persistent fitness launch, loss, ranking
    and update).  The labels are the base set's energies, forces and virials
    from the single-structure GPU path; the search starts from the base set
    perturbed by 0.05 with sigma 0.05."""
    import torch
    import workloads as W
    from paper_2603_01234_amd import engine
    fw = W.config3()
    spec = fw.specs[0]
    idx = [k for k in range(len(fw.systems)) if fw.family[k] == 0]
    base = fw.base_params[0]
    m0 = engine.Model.from_spec(spec, base.astype(np.float32))
    reps = []
    E_lab, F_lab, W_lab = [], [], []
    for k in idx:
        sysm = fw.systems[k]
        r = engine.Replica(m0, sysm.pos_f32(), sysm.types, sysm.box, sysm.pbc, skin=0.0)
        r.efv(per_bead_virial=False)
        E_lab.append(float(r.E_tot.cpu()[0]))
        F_lab.append(r.forces().astype(np.float64))
        W_lab.append(r.W_tot.cpu().numpy())
        reps.append(r)
    rng = np.random.default_rng(2603)
    mu0 = base + 0.05 * rng.normal(size=base.size)
    tr = engine.SnesTrainer(spec, mu0, 0.05, 64, reps, (E_lab, np.concatenate(F_lab), W_lab),
                            weights=(1.0, 1.0, 0.1, 1e-4, 1e-4), seed=7)
    best = tr.batch.autotune([(m, s) for m in range(8) for s in range(len(reps))])[0]
    tr.generation(cfg=best)                        # warm-up generation
    torch.cuda.synchronize()
    losses = []
    t0 = time.perf_counter()
    for _ in range(generations):
        tr.generation(cfg=best)
        losses.append(float(tr.loss.min().cpu()))
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / generations
    beads = 64 * sum(r.n for r in reps)
    out = {"workload": "SNES, 64 candidates x 1000 water-like structures (N log-uniform 32-1024), H = 30",
           "parameters": int(base.size), "generations": generations, "ms_per_generation": round(el * 1e3, 3),
           "bead_evals_per_s": round(beads / el, 1), "best_loss_per_generation": [round(x, 5) for x in losses],
           "note": "each generation: sample, derive the 64 candidates' tables, one persistent fitness launch, "
                   "loss/rank/update; the fitness call synchronises once"}
    tr.close()
    m0.close()
    return out


def labels_leg(steps: int = 100):
    """Constrained-MD label generation (Sec. II.C.1) with a synthetic two-type
    atomistic water model (H = 60, cutoffs 0.5/0.4 nm): the paper's 1536-atom /
    512-bead box and a 192,000-atom / 64,000-bead box, `steps` constrained NVE
    steps of 0.5 fs each, accumulating bead forces and virials every step."""
    import torch
    import workloads as W
    from paper_2603_01234_amd import engine
    spec = W.water_aa_spec(60)
    params = W.draw_params(spec, np.random.default_rng(2603))
    model = engine.Model.from_spec(spec, params)
    out = {"workload": "constrained NVE of atomistic water, beads = molecule centres of mass, dt 0.5 fs",
           "steps": steps}
    for n_side in (8, 40):
        sysm, gs = W.water_atomistic(np.random.SeedSequence(n_side), n_side, temperature=300.0)
        rep = engine.Replica(model, sysm.pos_f32(), sysm.types, sysm.box, sysm.pbc, skin=0.1, vel=sysm.vel)
        rep.efv(per_bead_virial=False)
        rep.constrained_labels(gs, 5, 0.5, sysm.masses, 300.0)          # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F, Wb, Wt = rep.constrained_labels(gs, steps, 0.5, sysm.masses, 300.0)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[f"atoms_{sysm.n}"] = {"beads": int(gs.size - 1), "ms_per_step": round(el * 1e3 / steps, 4),
                                  "atom_steps_per_s": round(sysm.n * steps / el, 1),
                                  "mean_bead_force_norm_eV_nm": round(float(np.linalg.norm(F, axis=1).mean()), 4),
                                  "corrected_pressure_GPa": round(float(np.trace(Wt)) / (3 * np.prod(sysm.box))
                                                                  * 0.1602176634, 4)}
        del rep
    model.close()
    return out


def batched_leg(reps: int = 3, plain_candidates: int = 2):
    """Fitness workload: 64 candidates x 2000 structures per family pair, one
    persistent launch per family (autotuned) against the plain loop of one
    nep_compute_efv call per (candidate, structure).  Labels are the base set's
    energies, forces and virials from the single-structure GPU path (they only
    set the residual values, not the work)."""
    import torch
    import workloads as W
    from paper_2603_01234_amd import binding as B
    from paper_2603_01234_amd import engine

    t_setup = time.perf_counter()
    fw = W.config3()
    fams = []
    for f in range(2):
        spec = fw.specs[f]
        idx = [k for k in range(len(fw.systems)) if fw.family[k] == f]
        models = [engine.Model.from_spec(spec, c.astype(np.float32)) for c in fw.candidates[f]]
        reps_f = []
        for k in idx:
            s = fw.systems[k]
            r = engine.Replica(models[0], s.pos_f32(), s.types, s.box, s.pbc, skin=0.0)
            r.build()
            reps_f.append(r)
        E_lab, F_lab, W_lab = [], [], []
        for r in reps_f:
            r.efv(per_bead_virial=False)
            E_lab.append(float(r.E_tot.cpu()[0]))
            F_lab.append(r.forces().astype(np.float64))
            W_lab.append(r.W_tot.cpu().numpy())
        fb = engine.FitnessBatch(models, reps_f)
        fb.set_labels(E_lab, np.concatenate(F_lab), W_lab)
        fams.append((spec, fb))
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup

    out = {"workload": "config3 fitness: 64 candidates (base + sigma 0.05 perturbations) x 2000 periodic "
                       "structures, N log-uniform 32-1024; 1000 water-like (1 type, rc 0.8/0.5 nm, density "
                       "x U(0.8,1.2)), 1000 C60-like monolayers (2 types, rc 2.0 nm); H = 30",
           "setup_s": round(t_setup, 1)}
    total_beads = 0
    t_batch = 0.0
    fam_out = []
    for f, (spec, fb) in enumerate(fams):
        work = fb.all_pairs()
        beads = sum(fb.replicas[s].n for _, s in work)
        # autotune on the first 8 candidates (all structures)
        sample = [(m, s) for (m, s) in work if m < 8]
        best, ms, tried, _ = fb.autotune(sample)
        t1 = time.perf_counter()
        _, _, _, hit = fb.autotune(sample)
        t_cached = time.perf_counter() - t1
        fb.evaluate(work, cfg=best)                      # warm-up at full size
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = fb.evaluate(work, cfg=best)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        t = float(np.median(times))
        rm = res["rmse"].cpu().numpy()
        # plain form: one nep_compute_efv (pack + fused + gather + reduce) per item
        pw = [(m, s) for (m, s) in work if m < plain_candidates]
        ws_plain = {}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pbeads = 0
        for m, s in pw:
            r = fb.replicas[s]
            sysc, nb = r.c_system(), r.c_neighbors()
            B.check(B.nep_compute_efv(fb.models[m].handle, sysc, nb, r.U.data_ptr(), r.F.data_ptr(), None,
                                      r.E_tot.data_ptr(), r.W_tot.data_ptr(), r.ws.data_ptr(), r.ws_bytes,
                                      torch.cuda.current_stream().cuda_stream))
            pbeads += r.n
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        fam_out.append({"family": ["water-like", "C60-like"][f], "items": len(work), "bead_evals": beads,
                        "batched_ms": round(t * 1e3, 2), "batched_bead_evals_per_s": round(beads / t, 1),
                        "plain_bead_evals_per_s": round(pbeads / t_plain, 1),
                        "plain_sample_items": len(pw),
                        "autotune": {"best": {"block": best.block, "order": best.order, "wg_per_cu": best.wg_per_cu,
                                              "schedule": ["given", "structure-major", "candidate-major",
                                                           "blocked-8"][best.schedule]},
                                     "search": [{"schedule": c.schedule, "order": c.order, "wg_per_cu": c.wg_per_cu,
                                                 "block": c.block, "ms_median_of_3": round(x, 3)}
                                                for c, x in zip(tried, ms)],
                                     "sample": "the first 8 candidates on every structure",
                                     "second_call_from_cache": hit,
                                     "second_call_ms": round(t_cached * 1e3, 3)},
                        "rmse_candidate0": [float(x) for x in rm[0]],
                        "rmse_candidate1": [float(x) for x in rm[1]]})
        total_beads += beads
        t_batch += t
    # whole-workload rates: both families, total bead-evaluations / total time
    t_plain_total = sum(x["bead_evals"] / x["plain_bead_evals_per_s"] for x in fam_out)
    out.update({"bead_evals_per_s": round(total_beads / t_batch, 1),
                "plain_bead_evals_per_s": round(total_beads / t_plain_total, 1),
                "speedup_vs_plain": round(t_plain_total / t_batch, 2),
                "families": fam_out})
    for _, fb in fams:
        for m in fb.models:
            m.close()
    return out


def served_leg(plain_requests: int = 2000):
    """Serving workload: 256 resident water-like replicas (500-20,000 beads,
    density x U(1.00, 1.25), config-0 weights, 300 K) and a Poisson trace of
    10-step requests at 2,000/s replayed in real time, through the continuous-
    batching server and through a plain FIFO loop of one nep_md_step call per
    request (first plain_requests requests of the same trace)."""
    import torch
    import workloads as W
    from paper_2603_01234_amd import engine

    sw = W.config4()
    model = engine.Model.from_spec(sw.spec, sw.params)
    n_req = len(sw.arrivals_s)
    steps = sw.steps_per_request

    def replay(submit, step, idle, n, t_first):
        t0 = time.perf_counter()
        i = 0
        while True:
            now = time.perf_counter() - t0
            while i < n and sw.arrivals_s[i] <= now:
                submit(i, t0 + float(sw.arrivals_s[i]))
                i += 1
            if idle():
                if i >= n:
                    break
                time.sleep(max(0.0, min(float(sw.arrivals_s[i]) - now, 1e-3)))
                continue
            step()
        return t0

    def serve(budget_frac):
        srv = engine.Server(model, sw.replicas, skin=0.1, dt=2.0, masses=[W.WATER_MASS], rebuild_every=10)
        full = sum(srv.footprint)
        t_setup = time.perf_counter()
        if budget_frac >= 1.0:
            for rid in range(len(sw.replicas)):          # everything fits: admit up front
                srv._admit(rid)
            srv.budget = max(srv.budget, srv.used)
        else:
            srv.budget = int(budget_frac * full)          # admission and eviction during the trace
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t_setup
        active_sizes = []

        def srv_step():
            active_sizes.append(len(srv.active) + min(len(srv.pending), srv.max_active))
            srv.tick()

        replay(lambda q, ta: srv.submit(q, int(sw.replica_of[q]), steps, ta), srv_step, srv.idle, n_req, 0)
        done = sorted(srv.done)
        warm = sw.warmup_requests
        lat = np.array([d[3] - d[2] for d in done[warm:]]) * 1e3
        meas = done[warm:]
        t_begin = min(d[2] for d in meas)
        t_end = max(d[3] for d in meas)
        bead_steps = sum(d[4] for d in meas)
        out = {"budget_fraction_of_all_replicas": budget_frac, "budget_bytes": int(srv.budget),
               "requests": n_req, "warmup_requests": warm, "ticks": srv.ticks,
               "mean_replicas_per_tick": round(float(np.mean(active_sizes)), 1),
               "admissions": srv.admissions, "evictions": srv.evictions,
               "bead_steps_per_s": round(bead_steps / (t_end - t_begin), 1),
               "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
               "setup_s": round(t_setup, 1)}
        return srv, out

    srv, served = serve(1.0)
    # saturated capacity: every replica active in every tick
    reps_all = [srv.replica(rid) for rid in range(len(sw.replicas))]
    stepper = srv.stepper
    stepper.step(reps_all)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ticks = 20
    for _ in range(ticks):
        stepper.step(reps_all)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    capacity = {"replicas_per_tick": len(reps_all), "ms_per_tick": round(el * 1e3 / ticks, 3),
                "bead_steps_per_s": round(sum(r.n for r in reps_all) * ticks / el, 1)}
    del srv, reps_all
    torch.cuda.empty_cache()
    _, served_half = serve(0.5)
    # plain FIFO loop over the first plain_requests requests, same arrival times
    reps = []
    for s in sw.replicas:
        r = engine.Replica(model, s.pos_f32(), s.types, s.box, s.pbc, skin=0.1, vel=s.vel)
        r.efv(per_bead_virial=False)
        reps.append(r)
    torch.cuda.synchronize()
    queue = []
    pdone = []

    def p_submit(q, ta):
        queue.append((q, ta))

    def p_step():
        q, ta = queue.pop(0)
        r = reps[int(sw.replica_of[q])]
        r.md(steps, 2.0, [W.WATER_MASS], rebuild_every=10)       # synchronises at its end
        pdone.append((q, ta, time.perf_counter(), r.n * steps))

    replay(p_submit, p_step, lambda: not queue, plain_requests, 0)
    pw = plain_requests // 10
    plat = np.array([d[2] - d[1] for d in pdone[pw:]]) * 1e3
    pt0 = min(d[1] for d in pdone[pw:])
    pt1 = max(d[2] for d in pdone[pw:])
    plain = {"requests": plain_requests, "warmup_requests": pw,
             "bead_steps_per_s": round(sum(d[3] for d in pdone[pw:]) / (pt1 - pt0), 1),
             "p50_ms": round(float(np.percentile(plat, 50)), 3), "p99_ms": round(float(np.percentile(plat, 99)), 3)}
    offered = float(np.mean([sw.replicas[int(k)].n for k in sw.replica_of])) * steps * n_req / float(sw.arrivals_s[-1])
    model.close()
    return {"workload": "config4 serving: 256 water-like replicas, N U{500..20000}, density x U(1.00,1.25), "
                        "config-0 weights, 300 K, skin 0.1 nm; Poisson 2000 req/s of 10 MD steps, "
                        "20,000 requests (first 1,000 warm-up)",
            "offered_bead_steps_per_s": round(offered, 1), "served": served, "served_half_budget": served_half,
            "capacity_all_replicas_active": capacity, "plain_fifo": plain,
            "throughput_ratio": round(served["bead_steps_per_s"] / plain["bead_steps_per_s"], 2),
            "note": "served: every replica resident; served_half_budget: an HBM budget of half the replicas' "
                    "footprint, so replicas are admitted and evicted (to host memory, lists included) during "
                    "the trace; capacity: every replica stepping in every tick"}


def network_engines_leg(rep, model, K, dt, masses, every, args):
    """The fused kernel with either network engine on the same state (the
    replica after the timed window, restored between the two runs): mean
    launch time over K steps and the steps' wall time."""
    from paper_2603_01234_amd import binding as B
    import torch
    snap = rep.snapshot()
    res = {}
    for eng in ("valu", "mfma"):
        rep.restore(snap)
        model.set_network(eng)
        B.nep_timing_begin(2 * K + 64, 0x1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep.md(K, dt, masses, rebuild_every=every, sort_every=args.sort_every)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms, launches = B.nep_timing_end()
        res[eng] = {"k_efv_main_avg_ms": round(ms[0] / max(launches[0], 1), 4),
                    "ms_per_step": round(wall * 1e3 / K, 4)}
    rep.restore(snap)
    model.set_network(args.network)
    res["note"] = ("both engines from the same snapshot of the timed state; the headline runs the engine in "
                   "config.network")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--pre-steps", type=int, default=-1,
                    help="untimed steps from the lattice before the warm-up (default: centre the timed window "
                         "on the 1000-step trajectory of the workload)")
    ap.add_argument("--split-steps", type=int, default=100,
                    help="steps of the run after the timed window that times every kernel class (0: none)")
    ap.add_argument("--no-full-run", action="store_true",
                    help="skip the separately timed whole 1000-step trajectory")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sort-every", type=int, default=100,
                    help="put the beads back into cell order every so many MD steps (0: never)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched fitness leg")
    ap.add_argument("--no-served", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-ensembles", action="store_true", help="skip the NVT / NPT / HNEMD leg")
    ap.add_argument("--no-snes", action="store_true", help="skip the SNES training-loop leg")
    ap.add_argument("--no-labels", action="store_true", help="skip the constrained label-generation leg")
    ap.add_argument("--network", choices=["valu", "mfma"], default="valu",
                    help="engine of the fused kernel's network (Eq. 2): vector ALUs or FP32 matrix cores")
    ap.add_argument("--no-network-legs", action="store_true",
                    help="skip the comparison of the two network engines on the timed state")
    ap.add_argument("--plain-skin-test", action="store_true",
                    help="MD rebuild gate: the two-largest-displacements test alone, without the pair test")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 256 MiB device copy (reference for the HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_2603_01234_amd import binding as B
    from paper_2603_01234_amd import engine

    torch.cuda.set_device(0)
    spec, params, system, opts = W.config1()
    model = engine.Model.from_spec(spec, params).set_network(args.network)
    masses = [W.WATER_MASS]
    dt, every = opts["dt"], opts["rebuild_every"]
    K = args.steps
    full_run = None
    if not args.no_full_run:
        # the whole workload as specified: 1000 steps from the lattice, timed as one
        fr = engine.Replica(model, system.pos_f32(), system.types, system.box, system.pbc,
                            skin=opts["skin"], vel=system.vel)
        fr.efv(per_bead_virial=False)
        fr.md(5, dt, masses, rebuild_every=every)          # first-launch costs, not part of the run
        fr = engine.Replica(model, system.pos_f32(), system.types, system.box, system.pbc,
                            skin=opts["skin"], vel=system.vel)
        fr.pair_test = not args.plain_skin_test
        fr.efv(per_bead_virial=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fr.md(opts["steps"], dt, masses, rebuild_every=every, sort_every=args.sort_every)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        full_run = {"steps": opts["steps"], "ms_per_step": round(el * 1e3 / opts["steps"], 4),
                    "bead_steps_per_s": round(system.n * opts["steps"] / el, 1),
                    "ns_per_day": round(opts["steps"] / el * dt * 86400 * 1e-6, 2),
                    "rebuilds": fr.n_rebuilds,
                    "note": "the whole 1000-step trajectory from the lattice, wall clock, virial every step"}
        del fr
    # the timed window: the central K steps of the same trajectory (pre-steps
    # and warm-up before it are untimed), so the window sees the trajectory's
    # typical state rather than the cold lattice it starts from
    pre = args.pre_steps if args.pre_steps >= 0 else max(0, (opts["steps"] - K) // 2 - args.warmup)
    rep = engine.Replica(model, system.pos_f32(), system.types, system.box, system.pbc,
                         skin=opts["skin"], vel=system.vel)
    rep.pair_test = not args.plain_skin_test
    rep.efv(per_bead_virial=False)          # lists + forces at t = 0
    if pre + args.warmup:
        rep.md(pre + args.warmup, dt, masses, rebuild_every=every, sort_every=args.sort_every)
    torch.cuda.synchronize()
    nR, nA = pair_counts(rep, spec)          # neighbours within the cutoffs at the start of the timed run
    print(f"bench: N={system.n}, mean neighbours within r_c: radial {nR.mean():.2f}, angular {nA.mean():.2f}",
          file=sys.stderr, flush=True)

    # row capacities with head-room for the density fluctuations of the run
    st = rep.status.cpu().tolist()
    rep._alloc_lists(max(rep.cap, int(st[1] * 1.5) + 16), max(rep.cap_A, int(st[2] * 1.5) + 16))
    rep.build()
    step_first = rep.step
    # fused-kernel launches before the window: the full run's (one evaluation
    # and 5 steps, then one evaluation and its steps), then this replica's
    # first evaluation and its steps so far (a run that overflows a row repeats
    # launches, so this is exact only for runs that never regrow)
    before = (0 if args.no_full_run else 1 + 5 + 1 + opts["steps"]) + 1 + step_first
    print(f"bench: timed window = MD steps {step_first}..{step_first + K - 1} of the trajectory "
          f"(k_efv_main dispatches {before + 1}..{before + K}, counting from 1)", file=sys.stderr, flush=True)
    counts = torch.zeros(2, dtype=torch.float64, device="cuda")
    Wtr = torch.zeros((max(K, 1), 9), dtype=torch.float64, device="cuda")
    # inside the timed region only the dominant kernel carries an event pair
    B.nep_timing_begin(2 * K + 64, 0x1)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    rb0 = rep.n_rebuilds
    rep.md(K, dt, masses, rebuild_every=every, pair_counts=counts, sort_every=args.sort_every, W_trace=Wtr)
    rebuilds = rep.n_rebuilds - rb0
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms, launches = B.nep_timing_end()
    elapsed = max(wall, gpu_ms / 1e3)
    # per-class split from a separate, shorter run that times every class
    K2 = min(K, args.split_steps)
    if K2 > 0:
        B.nep_timing_begin(8 * K2 + 64, 0xF)
        rb1 = rep.n_rebuilds
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rep.md(K2, dt, masses, rebuild_every=every, sort_every=args.sort_every)
        torch.cuda.synchronize()
        split_ms_step = (time.perf_counter() - t1) * 1e3 / K2
        ms_all, launches_all = B.nep_timing_end()
        rebuilds_split = rep.n_rebuilds - rb1
    value = system.n * K / elapsed
    ms_step = elapsed * 1e3 / K
    # algorithmic work of the timed region from the pairs the kernels evaluated
    tot_R, tot_A = counts.cpu().numpy().tolist()
    nR_run = np.full(system.n, tot_R / (K * system.n))
    nA_run = np.full(system.n, tot_A / (K * system.n))
    f_main, f_gather = algorithmic_flops(nR_run, nA_run, spec.n_hidden, spec.n_types)
    main_ms = ms[0] / max(launches[0], 1)
    achieved = f_main / (main_ms * 1e-3) / 1e12
    traffic = load_traffic(system.n)
    F_alg_bead = (f_main + f_gather) / system.n
    roofline = {
        "bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
        "kernel": "k_efv_main<1> (fused descriptor + network + angular pair forces)",
        "flops_per_launch": f_main, "avg_launch_ms": round(main_ms, 4),
    }
    kernels = None
    if K2 > 0:
        kernels = {name: {"avg_ms": round(ms_all[c] / max(launches_all[c], 1), 4), "launches": launches_all[c]}
                   for c, name in enumerate(["efv_main", "efv_gather", "neighbor_build", "kick_drift"])}
        kernels["split_run"] = {"steps": K2, "rebuilds": rebuilds_split, "ms_per_step": round(split_ms_step, 4),
                                "note": "every class timed; neighbor_build launches include the gated ones "
                                        "that found no rebuild due"}
    W_last = Wtr[K - 1].cpu().numpy().reshape(3, 3) if K > 0 else np.zeros((3, 3))
    vol = float(np.prod(system.box))
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "bead-steps/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "config1 CG water-like MD, 216,000 beads, NEP H=30 rc 0.8/0.5 nm, dt 2 fs, "
                               "rebuild every 10 steps, skin 0.1 nm",
                   "beads": system.n, "ns_per_day": round(K / elapsed * dt * 86400 * 1e-6, 2),
                   "mean_neighbours_radial_start": round(float(nR.mean()), 3),
                   "mean_neighbours_angular_start": round(float(nA.mean()), 3),
                   "mean_neighbours_radial_run": round(tot_R / (K * system.n), 3),
                   "mean_neighbours_angular_run": round(tot_A / (K * system.n), 3),
                   "row_capacity": [rep.cap, rep.cap_A],
                   "sort_every": args.sort_every,
                   "network": args.network,
                   "timed_steps": [step_first, step_first + K - 1],
                   "rebuilds_in_timed_steps": rebuilds,
                   "rebuild_gate": "two-largest displacements" if args.plain_skin_test else
                                   "two-largest displacements, then the pair test",
                   "virial": "per-bead and total virial every step (Eqs. 15-16)",
                   "virial_pressure_GPa_last_step": round(float(np.trace(W_last)) / (3 * vol) * 0.1602176634, 4),
                   "F_alg_per_bead_step": round(F_alg_bead, 1),
                   "path_tflops_alg": round(value * F_alg_bead / 1e12, 3)},
        "roofline": roofline,
    }
    if kernels is not None:
        out["kernels"] = kernels
    if not args.no_network_legs and K > 0:
        out["network_engines"] = network_engines_leg(rep, model, K, dt, masses, every, args)
    if full_run is not None:
        out["config"]["full_run"] = full_run
    if args.copy_calibration:
        # a plain elementwise kernel of known traffic: reads 256 MiB, writes 256 MiB
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.add(a, 1.0, out=b)
        torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, params, system, rep.positions().astype(np.float64))
    if not args.no_ensembles:
        print("bench: ensembles leg", file=sys.stderr, flush=True)
        out["ensembles"] = ensembles_leg(rep, dt, masses, every, sort_every=args.sort_every)
    model.close()
    if not args.no_batched:
        print("bench: batched fitness leg", file=sys.stderr, flush=True)
        out["batched"] = batched_leg()
    if not args.no_snes:
        print("bench: SNES leg", file=sys.stderr, flush=True)
        out["snes"] = snes_leg()
    if not args.no_labels:
        print("bench: label-generation leg", file=sys.stderr, flush=True)
        out["labels"] = labels_leg()
    if not args.no_served:
        print("bench: serving leg", file=sys.stderr, flush=True)
        out["served"] = served_leg()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
