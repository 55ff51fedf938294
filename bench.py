"""Throughput of the 3+1D Glasma CPIC hot path on one MI355X.

Headline workload (the method's plain SU(3) configuration): 512 x 64 x 64 lattice,
SU(3), a_T = 4 a_L, dt = a_L/2, two MV nuclei (mu = 0.5, sigma = 8 a_L, m = 0.2,
Lambda = 10/a_T), initial state built on the GPU.  One step = one leapfrog update of
every link and E field with the CPIC charge hop on every second step; observables
(T^{mu nu} slices, Gauss residual, energy) are reduced every 16 steps inside the
timed region (by the observing step, glasma_step_observe, on every 16th step of the timed
run).  Inputs are resident in HBM before timing starts.

The printed JSON line (scalars only, a few KB) reports site-updates/s of the FP64
single-event form (value), the roofline of its dominant kernel (the fused leapfrog step,
timed with HIP events on the library's stream), the FP32 single-event form, the FP32
batched form (64 events of N_z in {128,256,384} x N_T in {32,48,64}, 512 steps, HIP-graph
replay, autotuned tiling, event-averaged T^{mu nu}(z) on the device, and the relative error
of its observables against an FP64 run of the same events), the semi-implicit scheme on the headline
lattice, the differentiation form (gradient of the central-slab energy after 256 steps of
a 256 x 32 x 32 lattice, FP32 forward with checkpoints every 32 steps, FP64 reverse pass),
the local rest frame at the collision point after the collision (eps_loc from diagonalising
T^{mu nu}), nuclei of 8 colour sheets along the beam axis against the single sheet (GPU
initial conditions, energy between the receding nuclei), the approach of thin nuclei to the
boost-invariant Glasma at mid-rapidity, optionally the FP32-vs-FP64 precision study on the
2048 x 192 x 192 lattice, and the FP64 CPU oracle timed on the host.  Per-layer arrays and
tables go to the --detail file.
"""
import argparse
import hashlib
import json
import os
import re
import resource
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "leapfrog_su3_f64_512x64x64_counters.md")
KERNEL_SOURCES = ["step.hip", "stencil.h", "lattice.h", "group.h"]



# FP64 reunitarisation interval of the FP32 forms (in steps).  Measured against FP64 runs of
# the same inputs: every 4 steps instead of 8 halves the error of the observables (the 64
# batched events: per-event slices 1.7e-4 -> 9.9e-5; the 2048 x 192^2 lattice at step 256:
# 4.3e-5 -> 2.2e-5) and of the FP32-forward gradient (4.0e-5 -> 2.4e-5) for 1.5% of throughput.
FP32_REUNIT_EVERY = 4

def algorithmic_bytes_per_site_update(nc, fp, dt_over_aL):
    """Minimum HBM traffic of one site-update: read + write U (stored form: SU(2) 4 reals,
    SU(3) rows 0 and 1 = 12 reals) and E once, plus read + write of both charge populations
    on hop steps (a fraction dt/a_L of the steps)."""
    b = 8 if fp == 64 else 4
    r = 4 if nc == 2 else 12
    ng = nc * nc - 1
    return 2 * 3 * r * b + 2 * 3 * ng * b + 2 * 2 * ng * b * dt_over_aL


def kernel_source_hash():
    """sha256 (16 hex digits) of the step kernel's sources without their // comments and blank
    lines: a change of code, not of commentary, makes the committed counters stale."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2009_02044_amd", "csrc", f)) as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def counter_traffic():
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source (else None)."""
    try:
        txt = open(COUNTER_SUMMARY).read()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    hm = re.search(r"kernel_source_sha:\s*([0-9a-f]+)", txt)
    if not m or not hm or hm.group(1) != kernel_source_hash():
        return None
    return float(m.group(1))


def run_plain(w, fp, steps, warmup, obs_every=16, scheme=0, tol=1e-12):
    import torch
    import synth
    import paper_2009_02044_amd as pkg
    lat = pkg.Lattice(nc=w.nc, nz=w.nz, nt=w.nt, a_T=w.a_T, a_L=w.a_L, dt=w.dt, fp=fp,
                      reunit_every=FP32_REUNIT_EVERY if fp == 32 else 0, scheme=scheme, max_iter=200, tol=tol)
    rA, rB = synth.mv_charges(w.seed, w.nc, w.nt, w.mu, w.a_T)
    lat.init_mv(rA, rB, m_ir=w.m_ir, uv_cut=w.uv_cut, sigma=w.sigma, zA=w.zA, zB=w.zB)
    obs = lat.obs_buffer()
    torch.cuda.synchronize()
    lat.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    iters = []
    n_obs = 0
    while done < steps:
        n = min(obs_every, steps - done)
        if n == obs_every:
            # the last step of the chunk also reduces the observables of the state it starts
            # from (glasma_step_observe): observables every obs_every steps of the timed run
            if scheme == 1:
                lat.step(n - 1)
                lat.step_observe(1, obs)
                iters.append(lat.last_iterations)
            else:
                lat.step_observe(n, obs)
            n_obs += 1
        else:
            lat.step(n)
        if scheme == 1:
            iters.append(lat.last_iterations)
        done += n
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {"wall_s": wall, "ms_per_step": 1e3 * wall / steps, "observing_steps": n_obs,
           "site_updates_per_s": w.sites * steps / wall}
    if scheme == 0:
        # the dominant kernel alone (plain steps, no observables), HIP events recorded on the
        # library's stream; an even number of steps so that hop and no-hop steps are balanced
        st = lat.stream
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        nk = max(2, steps + (steps & 1))
        ev0.record(st)
        lat.step(nk)
        ev1.record(st)
        torch.cuda.synchronize()
        out["kernel_ms"] = ev0.elapsed_time(ev1) / nk
        out["kernel_steps"] = nk
    else:
        # per-step iteration counts of the timed run (last_iterations after each chunk)
        out["iterations_mean"] = float(np.mean(iters)) if iters else 0.0
    if n_obs == 0:
        lat.observe(obs)
    o = pkg.Lattice.unpack_obs(obs, w.nz)
    out.update({"gauss_rel": o["gauss_rel"], "energy": o["energy"], "unitarity": o["unitarity"]})
    return out


def run_rest_frame(w, after=224, every=32):
    """Local rest frame at the collision point of the headline lattice (Sec. 4): the nuclei
    (centres zB, zA, moving at the speed of light) meet at z_c = (zA + zB)/2 at
    t_c = (zA - zB)/2; from then on every `every` steps, eps_loc, the frame velocity, tau,
    eps_loc * tau and the pressure ratios 2 p_T / eps_loc, p_L / eps_loc at z_c (free
    streaming: eps_loc ~ 1/tau, 2 p_T = eps_loc, p_L ~ 0).  FP64, GPU observables."""
    import torch
    import synth
    import paper_2009_02044_amd as pkg
    lat = pkg.Lattice(nc=w.nc, nz=w.nz, nt=w.nt, a_T=w.a_T, a_L=w.a_L, dt=w.dt, fp=64)
    rA, rB = synth.mv_charges(w.seed, w.nc, w.nt, w.mu, w.a_T)
    lat.init_mv(rA, rB, m_ir=w.m_ir, uv_cut=w.uv_cut, sigma=w.sigma, zA=w.zA, zB=w.zB)
    z_c, t_c = 0.5 * (w.zA + w.zB), 0.5 * (w.zA - w.zB)
    kz = int(round(z_c / w.a_L))
    s_c = int(round(t_c / w.dt))
    obs = lat.obs_buffer()
    lat.step(s_c)
    rows = []
    for k in range(after // every):
        lat.step(every)
        lat.observe(obs)
        rf = lat.rest_frame(obs)
        torch.cuda.synchronize()
        o = pkg.Lattice.unpack_obs(obs, w.nz)
        el, v = (float(x) for x in rf[:, kz].cpu().numpy())
        eps, pL, pT, _ = (float(x) for x in o["tmunu_z"][:, kz])
        tau = (s_c + (k + 1) * every) * w.dt - t_c
        rows.append({"step": s_c + (k + 1) * every, "tau": tau, "eps_loc": el, "v": v,
                     "eps_loc_tau": el * tau, "2pT_over_eps_loc": 2 * pT / el, "pL_over_eps_loc": pL / el})
    return {"workload": w.name, "z_c": z_c, "t_c": t_c, "rows": rows}


def run_sheets(w, ns=8, after=128, every=64):
    """Nuclei with colour structure along the beam axis (ns independent sheets per
    nucleus, mu^2 / ns each) against the single sheet of the same width and a single
    sheet ns times thinner, on the headline lattice: time of the GPU initial conditions,
    H at t0, then, after the collision, eps at the collision point, the energy between
    the receding nuclei (|z - z_c| < t - t_c - 3 sigma) and H."""
    import torch
    import synth
    import paper_2009_02044_amd as pkg
    z_c, t_c = 0.5 * (w.zA + w.zB), 0.5 * (w.zA - w.zB)
    kz = int(round(z_c / w.a_L))
    s_c = int(round(t_c / w.dt))
    z = np.arange(w.nz) * w.a_L
    out = {"workload": w.name, "ns": ns, "z_c": z_c, "t_c": t_c}
    for key, n, sig in (("ns1", 1, w.sigma), ("ns%d" % ns, ns, w.sigma), ("ns1_thin", 1, w.sigma / ns)):
        lat = pkg.Lattice(nc=w.nc, nz=w.nz, nt=w.nt, a_T=w.a_T, a_L=w.a_L, dt=w.dt, fp=64)
        if n == 1:
            rA, rB = synth.mv_charges(w.seed, w.nc, w.nt, w.mu, w.a_T)
        else:
            rA, rB = synth.mv_sheet_charges(w.seed, w.nc, w.nt, w.mu, w.a_T, n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.init_mv(rA, rB, m_ir=w.m_ir, uv_cut=w.uv_cut, sigma=sig, zA=w.zA, zB=w.zB)
        torch.cuda.synchronize()
        init_ms = (time.perf_counter() - t0) * 1e3
        H0 = lat.observables()["energy"]
        obs = lat.obs_buffer()
        lat.step(s_c)
        rows = []
        for k in range(after // every):
            lat.step(every)
            lat.observe(obs)
            torch.cuda.synchronize()
            o = pkg.Lattice.unpack_obs(obs, w.nz)
            eps = o["tmunu_z"][0]
            tau = (s_c + (k + 1) * every) * w.dt - t_c
            inner = np.abs(z - z_c) < tau - 3 * w.sigma
            rows.append({"tau": tau, "eps_zc": float(eps[kz]),
                         "glasma_energy": float(eps[inner].sum() * w.a_L * w.a_T ** 2 * w.nt ** 2),
                         "H": float(o["energy"]), "gauss_rel": float(o["gauss_rel"])})
        out[key] = {"sheets": n, "sigma": sig, "init_ms": init_ms, "H0": H0, "rows": rows}
        del lat
    return out


def run_bi_limit(sigmas=(8.0, 4.0, 2.0, 1.0)):
    """Boost-invariant limit at mid-rapidity (Sec. 2, eqs. glasma_ic1/2): a lattice fine
    along z (a_T = 16 a_L, 96 x 32 x 32, dilute MV charges), nuclei of width sigma; after
    the collision, p_T(z_c) against eps_0 of the tau = 0+ boost-invariant fields of the
    same nuclei (glasma_bi_fields) and p_L / eps at z_c, for the leapfrog (dt = a_L/2)
    and the semi-implicit scheme (dt = a_L)."""
    import synth
    import paper_2009_02044_amd as pkg
    nc, nt, nz, aT = 3, 32, 96, 16.0
    m, mu, zA, zB = 0.8 / aT, 1.4 / aT, 72.0, 24.0
    rA, rB = synth.mv_charges(77, nc, nt, mu, aT)
    t_c, z_c = 0.5 * (zA - zB), int(0.5 * (zA + zB))
    out = {"lattice": [nz, nt, nt], "a_T": aT, "mu": mu, "m": m, "rows": []}
    for scheme, dt in ((0, 0.5), (1, 1.0)):
        for sig in sigmas:
            e0 = pkg.boost_invariant_fields(nc, nt, rA, rB, a_T=aT, m_ir=m)["eps0"]
            lat = pkg.Lattice(nc=nc, nz=nz, nt=nt, a_T=aT, a_L=1.0, dt=dt, fp=64, scheme=scheme,
                              max_iter=300, tol=1e-12)
            lat.init_mv(rA, rB, m_ir=m, uv_cut=0.0, sigma=sig, zA=zA, zB=zB)
            s_c = int(round(t_c / dt))
            per = int(round(2 / dt))
            lat.step(s_c)
            taus, pt, pl = [], [], []
            for k in range(10):
                lat.step(per)
                sl = lat.observables()["tmunu_z"]
                taus.append(2.0 * (k + 1))
                pt.append(float(sl[2][z_c] / e0))
                pl.append(float(sl[1][z_c] / sl[0][z_c]))
            i, j = int(np.argmax(pt)), int(np.argmin(pl))
            out["rows"].append({"scheme": "semi-implicit" if scheme else "leapfrog", "dt": dt, "sigma": sig,
                                "eps0": e0, "pT_over_eps0_max": pt[i], "tau_at_max": taus[i],
                                "pL_over_eps_min": pl[j], "tau_at_min": taus[j]})
            del lat
    return out


def run_rhic_profile(events, m_values=(0.2, 0.4, 0.8), T_fm=2.6):
    """Rapidity profile of the local rest-frame energy density in the RHIC set-up of Sec. 4
    (physunits.rhic_setup: SU(2), 2048 x 192^2 cells for a (6 fm)^3 box, sqrt(s) = 200 GeV,
    Q_s, mu, L, Lambda = 10 GeV from the printed relations): `events` MV events per IR
    regulator m, event-averaged T^{mu nu} diagonalised per layer on the GPU, eps_loc tau
    against eta_s in free streaming (physunits.rapidity_profile), Gaussian width sigma_eta."""
    import synth
    from paper_2009_02044_amd import physunits as pu
    out = {"events": events, "T_fm": T_fm, "rows": []}
    for m in m_values:
        su = pu.rhic_setup(m_GeV=m)
        t0 = time.perf_counter()
        charges = [synth.mv_charges(6000 + 100 * e, 2, su.nt, su.mu, su.a_T) for e in range(events)]
        r = pu.rapidity_profile(su, charges, T_fm, progress=lambda e, g: print(
            f"[rhic] m = {m} GeV: event {e + 1}/{events} done, Gauss {g:.1e}", file=sys.stderr, flush=True))
        wall = time.perf_counter() - t0
        eta, f = r["eta"], r["eps_loc_tau"]
        out["rows"].append({"m_GeV": m, "sigma_eta": r["sigma_eta"], "eta_max": float(np.abs(eta).max()),
                            "sigma_cells": su.sigma, "mu_lat": su.mu, "m_lat": su.m_ir, "a_T": su.a_T,
                            "steps": r["steps"], "wall_s": wall, "gauss_rel_max": r["gauss_rel_max"],
                            "profile_eta": [float(x) for x in eta[::16]],
                            "profile_eps_loc_tau": [float(x) for x in f[::16]]})
        print(f"[bench] RHIC 200 GeV, m = {m} GeV, {events} events: sigma_eta {r['sigma_eta']:.2f} "
              f"(|eta| <= {np.abs(eta).max():.2f}), {wall:.1f} s", file=sys.stderr, flush=True)
    return out


def run_batched(steps, warmup, graph_chunk=16, n_grid=64, compare_fp64=True):
    """64 events, SU(3) FP32: autotuned tiling, then the timed run (HIP-graph replay); the
    event-averaged T^{mu nu}(z) on the device (glasma_batch_observe: per N_z class and on a
    common z / N_z grid of n_grid bins).  With compare_fp64 the same 64 events (same initial
    conditions) run the same number of steps in FP64 and the FP32 observables are compared
    with them: the error of the FP32 form at the step count it is timed at."""
    import torch
    import synth
    import paper_2009_02044_amd as pkg
    from paper_2009_02044_amd import _lib
    evs = synth.batched_events()
    shapes = [(w.nz, w.nt) for w in evs]

    def make(fp):
        b = pkg.Batch(3, shapes, a_T=4.0, a_L=1.0, dt=0.5, fp=fp, reunit_every=FP32_REUNIT_EVERY if fp == 32 else 0)

        def init():
            for w, lat in zip(evs, b.events):
                rA, rB = synth.mv_charges(w.seed, 3, w.nt, w.mu, w.a_T)
                lat.init_mv(rA, rB, m_ir=w.m_ir, uv_cut=w.uv_cut, sigma=w.sigma, zA=w.zA, zB=w.zB)
            b.stream.synchronize()
        return b, init

    b, init = make(32)
    init()
    tune = b.autotune(steps=4)
    init()
    b.run(warmup, graph_chunk=0)
    b.stream.synchronize()
    t0 = time.perf_counter()
    b.run(steps, graph_chunk=graph_chunk)
    b.stream.synchronize()
    wall = time.perf_counter() - t0
    r32 = b.observe(n_grid, per_event=True)
    b.stream.synchronize()
    pe32 = r32["per_event"].cpu().numpy()
    out = {"site_updates_per_s": b.sites * steps / wall, "ms_per_step": 1e3 * wall / steps, "sites": b.sites, "events": len(evs),
           "steps": warmup + steps, "timed_steps": steps, "tiling": tune["chosen"],
           "classes": b.classes(), "n_grid": n_grid,
           "tmunu_z_event_avg_grid": r32["grid"].cpu().numpy().tolist(),
           "tmunu_z_event_avg_by_nz": {str(k): v.cpu().numpy().tolist() for k, v in r32["class"].items()}}
    nz_list = [w.nz for w in evs]
    g32 = [o["gauss_rel"] for o in (b.events[e].observables() for e in range(len(evs)))]
    out["gauss_rel_max"] = float(max(g32))
    del b, r32
    torch.cuda.empty_cache()
    if not compare_fp64:
        return out
    b64, init64 = make(64)
    init64()
    b64.run(warmup + steps, graph_chunk=graph_chunk)
    r64 = b64.observe(n_grid, per_event=True)
    b64.stream.synchronize()
    pe64 = r64["per_event"].cpu().numpy()
    # per-event relative errors of the slices (max over z / max |FP64 slice|) and totals
    rows, off = [], 0
    for e, nz in enumerate(nz_list):
        a = pe32[off:off + 4 * nz].reshape(4, nz)
        c = pe64[off:off + 4 * nz].reshape(4, nz)
        row = {}
        for q, name in enumerate(("eps", "pL", "pT")):
            row[name + "_slices"] = float(np.abs(a[q] - c[q]).max() / np.abs(c[q]).max())
            row[name + "_total"] = float(abs(a[q].sum() - c[q].sum()) / abs(c[q].sum()))
        hs = pe32[off + 4 * nz], pe64[off + 4 * nz]
        row["H"] = float(abs(hs[0] - hs[1]) / abs(hs[1]))
        rows.append(row)
        off += 4 * nz + _lib.OBS_NSCALARS
    keys = list(rows[0])
    err = {k: {"max": float(max(r[k] for r in rows)), "median": float(np.median([r[k] for r in rows]))} for k in keys}
    grid32 = np.array(out["tmunu_z_event_avg_grid"])
    grid64 = r64["grid"].cpu().numpy()
    for q, name in enumerate(("eps", "pL", "pT")):
        err["event_avg_grid_" + name] = float(np.abs(grid32[q] - grid64[q]).max() / np.abs(grid64[q]).max())
    out["fp32_vs_fp64_same_events"] = err
    out["fp32_vs_fp64_per_event"] = rows
    del b64, r64
    torch.cuda.empty_cache()
    return out


def run_adjoint(w, steps, every, fp=32):
    """Differentiation form: forward pass with a checkpoint every `every` steps, then the
    reverse pass (segment recompute + reverse kernels) for the gradient of the central
    16-layer energy with respect to E0 and the per-cell charge amplitudes."""
    import torch
    import synth
    import paper_2009_02044_amd as pkg
    lat = pkg.Lattice(nc=w.nc, nz=w.nz, nt=w.nt, a_T=w.a_T, a_L=w.a_L, dt=w.dt, fp=fp,
                      reunit_every=FP32_REUNIT_EVERY if fp == 32 else 0)
    rA, rB = synth.mv_charges(w.seed, w.nc, w.nt, w.mu, w.a_T)
    lat.init_mv(rA, rB, m_ir=w.m_ir, uv_cut=w.uv_cut, sigma=w.sigma, zA=w.zA, zB=w.zB)
    s0 = lat.get_state_device()
    work = lat.adjoint_work(steps, every)
    z0, z1 = w.nz // 2 - 8, w.nz // 2 + 8
    times = []
    for rep in range(2):                       # the first pass warms up
        lat.set_state_device(s0["U"], s0["E"], s0["rhoA"], s0["rhoB"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.adjoint_forward(steps, every, work)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g = lat.adjoint_backward(z0, z1, work)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times.append((t1 - t0, t2 - t1))
    fwd, bwd = times[-1]
    return {"site_updates_per_s": w.sites * steps / (fwd + bwd), "forward_s": fwd, "backward_s": bwd,
            "backward_over_forward": bwd / fwd, "workload": w.name, "steps": steps, "ckpt_every": every,
            "forward_dtype": "f32" if fp == 32 else "f64", "adjoint_dtype": "f64",
            "work_bytes": int(work.numel()), "loss": g["L"],
            "grad_norm_E0": float(g["dE0"].norm()), "grad_norm_ampA": float(g["dampA"].norm())}


def run_precision(w, steps, every=256):
    """Precision form: FP32 storage and arithmetic with FP64 reunitarisation every
    FP32_REUNIT_EVERY steps,
    against the FP64 GPU run from the same initial state; relative errors of the per-layer
    eps, p_L, p_T and of their totals at intervals of `every` steps."""
    import torch
    import synth
    import paper_2009_02044_amd as pkg
    rA, rB = synth.mv_charges(w.seed, w.nc, w.nt, w.mu, w.a_T)
    series = {}
    for fp in (64, 32):
        lat = pkg.Lattice(nc=w.nc, nz=w.nz, nt=w.nt, a_T=w.a_T, a_L=w.a_L, dt=w.dt, fp=fp,
                          reunit_every=FP32_REUNIT_EVERY if fp == 32 else 0)
        lat.init_mv(rA, rB, m_ir=w.m_ir, uv_cut=w.uv_cut, sigma=w.sigma, zA=w.zA, zB=w.zB)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        obs = []
        for k in range(steps // every):
            lat.step(every)
            obs.append(lat.observables())
            print(f"[bench] precision fp{fp}: step {(k + 1) * every}", file=sys.stderr, flush=True)
        series[fp] = {"obs": obs, "wall_s": time.perf_counter() - t0}
        del lat
        torch.cuda.empty_cache()
    rows = []
    for k in range(steps // every):
        a, b = series[32]["obs"][k], series[64]["obs"][k]
        row = {"step": (k + 1) * every}
        for q, name in enumerate(("eps", "pL", "pT")):
            s32, s64 = a["tmunu_z"][q], b["tmunu_z"][q]
            row[f"{name}_slices_max_rel"] = float(np.abs(s32 - s64).max() / np.abs(s64).max())
            row[f"{name}_total_rel"] = float(abs(s32.sum() - s64.sum()) / abs(s64.sum()))
        row["gauss_rel_fp32"] = a["gauss_rel"]
        row["unitarity_fp32"] = a["unitarity"]
        rows.append(row)
    return {"workload": w.name, "lattice": [w.nz, w.nt, w.nt], "steps": steps, "reunit_every": FP32_REUNIT_EVERY,
            "fp64_wall_s": series[64]["wall_s"], "fp32_wall_s": series[32]["wall_s"], "rows": rows}


def memory_ceiling(nbytes=1 << 30, reps=10):
    """What the memory system delivers on this device, as a ceiling for the HBM fractions: a
    device-to-device copy of 1 GiB (torch's copy kernel; read + write bytes), HIP events on the
    current stream, best of reps."""
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        ev0.record()
        y.copy_(x)
        ev1.record()
        torch.cuda.synchronize()
        best = min(best, ev0.elapsed_time(ev1))
    del x, y
    return {"copy_GBps": 2 * nbytes / (best * 1e-3) / 1e9, "bytes": nbytes}


def cpu_baseline(w, budget_s=20.0):
    """The FP64 oracle on a bounded sample of the same workload: a 64-layer slab of the
    beam axis at the full transverse size, stepped until ~budget_s of CPU time."""
    import synth
    from oracle import lattice, init_mv
    nz = 64
    ws = synth.Workload("slab", nc=w.nc, nz=nz, nt=w.nt, a_T=w.a_T, a_L=w.a_L, dt=w.dt, mu=w.mu,
                        sigma=w.sigma, m_ir=w.m_ir, uv_cut=w.uv_cut, seed=w.seed)
    p = lattice.Params(ws.nc, ws.a_T, ws.a_L, ws.dt)
    mv = init_mv.MVParams(ws.m_ir, ws.uv_cut, ws.sigma, ws.zA, ws.zB)
    rA, rB = synth.mv_charges(ws.seed, ws.nc, ws.nt, ws.mu, ws.a_T)
    st, _ = init_mv.initial_state(rA, rB, nz, p, mv)
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    n = 0
    while True:
        st = lattice.leapfrog_step(st)
        n += 1
        if time.perf_counter() - t0 > budget_s or n >= 8:
            break
    wall = time.perf_counter() - t0
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    return {"value": ws.sites * n / wall, "unit": "site-updates/s",
            "cores": max(1, int(round(cpu / wall))), "kind": "oracle",
            "sample": f"{n} leapfrog steps of a {nz}x{ws.nt}x{ws.nt} slab of the headline "
                      f"lattice (SU({ws.nc}), FP64 NumPy)",
            "host_cpus": os.cpu_count(), "cpu_model": cpu_model(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def scalars(d, keep):
    """The entries of d named in keep whose values are numbers or short strings."""
    return {k: d[k] for k in keep if k in d and isinstance(d[k], (int, float, str, type(None)))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=256)
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-batched-fp64", action="store_true",
                    help="skip the FP64 run of the batched events (the at-fixed-error comparison)")
    ap.add_argument("--no-semi", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=512)
    ap.add_argument("--semi-steps", type=int, default=8)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-rest-frame", action="store_true")
    ap.add_argument("--no-sheets", action="store_true")
    ap.add_argument("--no-bi-limit", action="store_true")
    ap.add_argument("--detail", default=os.path.join("results", "bench_detail.json"),
                    help="file for the full results (per-layer arrays, tables); the printed line holds scalars")
    ap.add_argument("--rhic-profile", type=int, default=0,
                    help="also run the RHIC 200 GeV rapidity-profile study with this many events per m")
    ap.add_argument("--precision-study", action="store_true",
                    help="also run the FP32-vs-FP64 comparison on the 2048 x 192 x 192 lattice (minutes)")
    ap.add_argument("--precision-steps", type=int, default=2048)
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the bounded FP32-vs-FP64 run of the 2048 x 192 x 192 precision workload "
                         "(256 steps; --precision-study runs the full length)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device to device (scale for HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        x = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 1 << 30}))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU: this build has no multi-GPU path (the z-slab sharding "
              "is a design only); run it with --gpus 1", file=sys.stderr)
        print(json.dumps({"error": "one GPU only; --gpus must be 1", "n_gpus": args.gpus}))
        sys.exit(2)
    import synth
    w = synth.PLAIN_SU3
    r64 = run_plain(w, 64, args.steps, args.warmup)
    print(f"[bench] fp64 {w.name}: {r64['site_updates_per_s']:.3e} site-updates/s, "
          f"kernel {r64['kernel_ms']:.3f} ms", file=sys.stderr, flush=True)
    forms, detail = {}, {"fp64_plain": r64}
    if not args.no_fp32:
        r32 = run_plain(w, 32, args.steps, args.warmup)
        b32 = algorithmic_bytes_per_site_update(3, 32, w.dt / w.a_L)
        forms["fp32_plain"] = {
            "site_updates_per_s": r32["site_updates_per_s"], "kernel_ms": r32["kernel_ms"],
            "kernel_site_updates_per_s": w.sites / (r32["kernel_ms"] * 1e-3),
            "hbm_frac": b32 * w.sites / (r32["kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "gauss_rel": r32["gauss_rel"], "unitarity": r32["unitarity"]}
        detail["fp32_plain"] = r32
        print(f"[bench] fp32 {w.name}: {r32['site_updates_per_s']:.3e} site-updates/s",
              file=sys.stderr, flush=True)
    if not args.no_batched:
        rb = run_batched(args.batched_steps, 8, compare_fp64=not args.no_batched_fp64)
        bb = algorithmic_bytes_per_site_update(3, 32, 0.5)
        rb["hbm_frac"] = bb * rb["site_updates_per_s"] / 1e9 / HBM_PEAK_GBS
        rb["vs_fp64_plain"] = rb["site_updates_per_s"] / r64["site_updates_per_s"]
        detail["fp32_batched"] = rb
        fb = scalars(rb, ("site_updates_per_s", "ms_per_step", "hbm_frac", "vs_fp64_plain", "sites", "events",
                          "steps", "gauss_rel_max"))
        fb["tiling"] = rb["tiling"]
        if "fp32_vs_fp64_same_events" in rb:
            e = rb["fp32_vs_fp64_same_events"]
            fb["rel_err_vs_fp64_max_over_events"] = {k: round(v["max"], 9) for k, v in e.items()
                                                     if isinstance(v, dict)}
            fb["rel_err_event_avg"] = {k[len("event_avg_grid_"):]: round(v, 9) for k, v in e.items()
                                       if k.startswith("event_avg_grid_")}
        forms["fp32_batched"] = fb
        print(f"[bench] fp32 batched 64 events: {rb['site_updates_per_s']:.3e} site-updates/s "
              f"({rb['vs_fp64_plain']:.2f}x fp64 plain)", file=sys.stderr, flush=True)
    if not args.no_semi:
        for dt in (0.5, 1.0):
            ws = synth.Workload(w.name, nc=3, nz=w.nz, nt=w.nt, dt=dt, mu=w.mu, sigma=w.sigma,
                                uv_cut=w.uv_cut, seed=w.seed)
            rs = run_plain(ws, 64, args.semi_steps, 1, obs_every=4, scheme=1, tol=1e-12)
            key = f"semi_implicit_fp64_dt{dt}"
            forms[key] = scalars(rs, ("site_updates_per_s", "ms_per_step", "iterations_mean", "gauss_rel"))
            forms[key]["tol"] = 1e-12
            detail[key] = rs
            print(f"[bench] semi-implicit dt={dt}: {rs['site_updates_per_s']:.3e} site-updates/s, "
                  f"{rs['iterations_mean']:.1f} iterations", file=sys.stderr, flush=True)
        # the same run at dt = a_L in FP32 storage and arithmetic (fixed point iterated to 1e-6,
        # about FP32 resolution); its final field energy against the FP64 run's
        rs32 = run_plain(ws, 32, args.semi_steps, 1, obs_every=4, scheme=1, tol=1e-6)
        key = "semi_implicit_fp32_dt1.0"
        forms[key] = scalars(rs32, ("site_updates_per_s", "ms_per_step", "iterations_mean", "gauss_rel"))
        forms[key]["tol"] = 1e-6
        forms[key]["energy_rel_err_vs_fp64"] = abs(rs32["energy"] - detail["semi_implicit_fp64_dt1.0"]["energy"]) / abs(
            detail["semi_implicit_fp64_dt1.0"]["energy"])
        detail[key] = rs32
        print(f"[bench] semi-implicit dt=1.0 fp32: {rs32['site_updates_per_s']:.3e} site-updates/s, "
              f"{rs32['iterations_mean']:.1f} iterations, energy vs fp64 {forms[key]['energy_rel_err_vs_fp64']:.1e}",
              file=sys.stderr, flush=True)
    if not args.no_adjoint:
        wa = synth.ADJOINT_SU3
        ra = run_adjoint(wa, wa.steps, 32)
        forms["adjoint_fp32_fwd_fp64_rev"] = scalars(ra, ("site_updates_per_s", "forward_s", "backward_s",
                                                          "backward_over_forward", "steps", "ckpt_every"))
        detail["adjoint"] = ra
        print(f"[bench] adjoint {wa.name}: forward {ra['forward_s']:.3f} s, backward {ra['backward_s']:.3f} s",
              file=sys.stderr, flush=True)
    if not args.no_rest_frame:
        detail["rest_frame_collision_point"] = rf = run_rest_frame(w)
        r = rf["rows"][-1]
        forms["rest_frame_collision_point"] = {k: r[k] for k in ("tau", "eps_loc_tau", "2pT_over_eps_loc",
                                                                  "pL_over_eps_loc")}
        print(f"[bench] rest frame at z_c: tau {r['tau']:.0f}, eps_loc tau {r['eps_loc_tau']:.3e}, "
              f"2pT/eps_loc {r['2pT_over_eps_loc']:.3f}, pL/eps_loc {r['pL_over_eps_loc']:.3f}",
              file=sys.stderr, flush=True)
    if not args.no_sheets:
        detail["colour_sheets"] = r = run_sheets(w)
        one, many, thin = r["ns1"], r["ns%d" % r["ns"]], r["ns1_thin"]
        a, b, c = one["rows"][-1], many["rows"][-1], thin["rows"][-1]
        forms["colour_sheets"] = {"ns": r["ns"], "init_ms": many["init_ms"],
                                  "glasma_energy_ratio_vs_one_sheet": b["glasma_energy"] / a["glasma_energy"]}
        print(f"[bench] {r['ns']} colour sheets: init {many['init_ms']:.1f} ms (1 sheet {one['init_ms']:.1f} ms); "
              f"at tau {a['tau']:.0f} glasma energy {b['glasma_energy']:.4g} vs {a['glasma_energy']:.4g} (1 sheet) "
              f"and {c['glasma_energy']:.4g} (1 sheet, sigma/{r['ns']})", file=sys.stderr, flush=True)
    if not args.no_bi_limit:
        detail["boost_invariant_limit"] = r = run_bi_limit()
        forms["boost_invariant_limit"] = {f"sigma{row['sigma']:g}": round(row["pT_over_eps0_max"], 4)
                                          for row in r["rows"] if row["scheme"] == "semi-implicit"}
        for row in r["rows"]:
            if row["scheme"] == "semi-implicit":
                print(f"[bench] boost-invariant limit, semi-implicit, sigma {row['sigma']:g}: "
                      f"max p_T/eps_0 {row['pT_over_eps0_max']:.3f}, min p_L/eps {row['pL_over_eps_min']:+.3f}",
                      file=sys.stderr, flush=True)
    if args.rhic_profile > 0:
        detail["rhic200_rapidity_profile"] = run_rhic_profile(args.rhic_profile)
    if args.precision_study or not args.no_precision:
        wp = synth.PRECISION_SU3
        full = args.precision_study
        rp = run_precision(wp, args.precision_steps if full else 256, every=256 if full else 128)
        detail["precision_fp32_vs_fp64"] = rp
        keys = ("eps_slices_max_rel", "eps_total_rel", "pL_slices_max_rel", "pL_total_rel", "pT_slices_max_rel",
                "pT_total_rel", "gauss_rel_fp32")
        forms["precision_fp32_vs_fp64"] = {
            "workload": wp.name, "lattice": rp["lattice"], "reunit_every": rp["reunit_every"],
            "fp32_wall_s": round(rp["fp32_wall_s"], 2), "fp64_wall_s": round(rp["fp64_wall_s"], 2),
            "rows": [{"step": r["step"], **{k: float(f"{r[k]:.3g}") for k in keys}} for r in rp["rows"]]}
        last = rp["rows"][-1]
        print(f"[bench] precision form {wp.name}, step {last['step']}: eps / p_L / p_T slices within "
              f"{last['eps_slices_max_rel']:.2e} / {last['pL_slices_max_rel']:.2e} / {last['pT_slices_max_rel']:.2e} "
              f"of FP64 (FP32 {rp['fp32_wall_s']:.1f} s, FP64 {rp['fp64_wall_s']:.1f} s)", file=sys.stderr, flush=True)
    bpsu = algorithmic_bytes_per_site_update(3, 64, w.dt / w.a_L)
    launch_bytes = bpsu * w.sites
    achieved = launch_bytes / (r64["kernel_ms"] * 1e-3) / 1e9
    ceil = memory_ceiling()
    print(f"[bench] memory ceiling: device copy {ceil['copy_GBps']:.0f} GB/s",
          file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w)
        print(f"[bench] cpu oracle: {cpu['value']:.3e} site-updates/s", file=sys.stderr, flush=True)
    line = {
        "metric": "site-updates/s + HBM GB/s fraction; FP32-batched vs FP64-plain at fixed error",
        "value": r64["site_updates_per_s"],
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (MV charges, seeded)",
        "config": {"workload": w.name, "form": "plain SU(3) FP64 leapfrog + CPIC, single event", "nc": 3,
                   "lattice": [w.nz, w.nt, w.nt], "a_T": w.a_T, "dt": w.dt, "scheme": "leapfrog",
                   "obs_every": 16, "observing_steps_timed": r64["observing_steps"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic(),
                     "kernel": "k_leapfrog<Su3<double>,double,hop,xs=true>", "kernel_ms": r64["kernel_ms"],
                     "kernel_site_updates_per_s": w.sites / (r64["kernel_ms"] * 1e-3),
                     "bytes_per_site_update": bpsu,
                     "bytes_row": "SU(3) FP64, links stored by 2 rows (12 reals): 2(288 + 192) + 128 x dt/a_L",
                     "bytes_per_launch": launch_bytes,
                     "copy_ceiling_GBps": ceil["copy_GBps"],
                     "frac_of_copy_ceiling": achieved / ceil["copy_GBps"]},
        "checks": {"gauss_rel": r64["gauss_rel"], "unitarity": r64["unitarity"]},
        "forms": forms,
        "cpu_baseline": cpu,
        "detail_file": args.detail,
    }
    if args.detail:
        d = os.path.dirname(args.detail)
        if d:
            os.makedirs(d, exist_ok=True)
        with open(args.detail, "w") as fh:
            json.dump({"line": line, "detail": detail}, fh)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
