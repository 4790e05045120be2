"""Throughput benchmark: energy + force atom-steps/s on one MI355X.

A step is one pass of the whole hot path on GPU-resident state, run by the
native MD engine (nnp_md_run: the steps are enqueued in one go and the host
waits once, at the end): integrator half steps, the on-device rebuild
decision, neighbour list build (cell list) when due, AEV, species networks,
AEV adjoint, force gather and the float64 structure energy (summed on every
step).

Default workload: the large periodic water box, 33,333 rigid-geometry waters
(99,999 atoms, 1.0 g/cm^3, L = 99.905 A), velocity Verlet at dt = 0.5 fs
from 300 K Maxwell-Boltzmann velocities, neighbour list with a 0.5 A skin
rebuilt every 20 steps and earlier when the Verlet-list bound requires it.
The headline value is the FP32 form (the paper's precision); the BF16-MLP
form runs beside it.  ``--config 2`` runs the 4,500-atom box (no skin, list
rebuilt every step) and ``--config 3`` the 23,000-atom organic box (energy
and forces only, no dynamics, with both forms' errors against the FP64
oracle).  ``--config 4`` is the serving form (``--serving-sweep`` sweeps the
request rate).

Prints one JSON line.  Inputs are synthetic and seeded; weights are random
(Glorot-uniform, seed 123456).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X_PEAK = {"hbm_GBs": 8000.0, "fp32_TFLOPs": 157.3, "bf16_TFLOPs": 2500.0}


def mlp_flops_per_atom(widths):
    fwd = sum(2 * widths[l] * widths[l + 1] for l in range(len(widths) - 1))
    adj = sum(2 * widths[l] * widths[l + 1] for l in range(len(widths) - 2))   # head adjoint is elementwise
    return fwd, adj


def fused_tile_rows(n_atoms, precision, nets=1):
    """Rows per tile of the fused network kernel (as the library chooses them):
    64 only for the BF16 ensemble from 48 Ki atoms, else at most 32."""
    tm = 64 if n_atoms >= 48 * 1024 else (32 if n_atoms >= 12 * 1024 else 16)
    return tm if (precision == "bf16" and nets > 1) else min(tm, 32)


_MASKS = {}


def species_masks(w, spec):
    """Per atom: bits 0-7 the species within Rc_R, 8-15 those within Rc_A."""
    key = (w.name, w.n_atoms)
    if key in _MASKS:
        return _MASKS[key]
    from scipy.spatial import cKDTree
    N = w.n_atoms
    x = w.pos.astype(np.float64)
    kw = {}
    if w.box is not None:
        L = np.asarray(w.box, dtype=np.float64)
        x = np.mod(x, L)
        x[x >= L] = 0.0
        kw["boxsize"] = L
    tree = cKDTree(x, **kw)
    sp = w.species.astype(np.int64)
    mask = np.zeros(N, dtype=np.int64)
    for r, shift in ((spec.rc_r, 0), (spec.rc_a, 8)):
        pr = tree.query_pairs(r, output_type="ndarray")
        if len(pr):
            np.bitwise_or.at(mask, pr[:, 0], 1 << (shift + sp[pr[:, 1]]))
            np.bitwise_or.at(mask, pr[:, 1], 1 << (shift + sp[pr[:, 0]]))
    _MASKS[key] = mask
    return mask


def active_features(m, ns):
    """Features of the blocks a species mask can make non-zero."""
    blocks = sum(1 for q in range(ns) if (m >> q) & 1)
    blocks += sum(2 for q in range(ns) for u in range(q, ns) if (m >> (8 + q)) & (m >> (8 + u)) & 1)
    return 16 * blocks


def mlp_useful_flops(w, spec, precision, nets=1):
    """FLOP of one launch of the fused networks counting only the first
    layer's products (forward and adjoint) over the feature blocks that some
    atom of each species tile can have non-zero, as the kernel runs them: a
    species' 16 radial features when it occurs within Rc_R of an atom of the
    tile, a species pair's 32 angular features when both occur within Rc_A.
    Returns (useful FLOP, dense FLOP, mean active features per atom)."""
    N, ns = w.n_atoms, spec.n_species
    mask = species_masks(w, spec)
    widths = spec.widths
    n1, D = widths[1], spec.aev_dim
    fwd, adj = mlp_flops_per_atom(widths)
    dense = (fwd + adj) * nets * N
    tm = fused_tile_rows(N, precision, nets)
    useful, feats = 0.0, 0.0
    for s in range(ns):
        idx = np.nonzero(w.species == s)[0]
        for t0 in range(0, len(idx), tm):
            F = active_features(int(np.bitwise_or.reduce(mask[idx[t0:t0 + tm]])), ns)
            rows = len(idx[t0:t0 + tm])
            feats += F * rows
            f_fwd = fwd - 2 * D * n1 + 2 * F * n1
            f_adj = adj - 2 * n1 * D + 2 * n1 * F
            useful += nets * (f_fwd + f_adj) * rows
    return useful, dense, feats / max(N, 1)


# one kernel per timed stage where the roofline is reported
STAGE_KERNEL = {("mlp", True): "k_mlp_fused", ("mlp", False): "k_gemm_* chain", ("aev", True): "k_aev_fwd",
                ("aev", False): "k_aev_fwd", ("aev_adjoint", True): "k_aev_bwd",
                ("aev_adjoint", False): "k_aev_bwd", ("forces", True): "k_force_gather",
                ("forces", False): "k_force_gather"}
STAGE_SOURCE = {"mlp": "mlp_fused.hip", "aev": "aev.hip", "aev_adjoint": "aev.hip", "forces": "forces.hip",
                "neighbors": "neighbors.hip"}


def stage_bytes(stage, N, P, precision, D, Fg=None):
    """Algorithmic HBM bytes of one launch: every input read once, every
    output written once (N atoms, P list pairs, D features; the adjoint reads
    dE/dAEV only for the Fg features per atom its environment can make
    non-zero, D when not given)."""
    Fg = D if Fg is None else Fg
    feat = 2 if precision == "bf16" else 4       # feature rows handed to the networks
    nl = 4 * (N + 1) + 7 * P                     # row_ptr, col (int32), shift (3 x int8)
    atoms = 20 * N                               # position, species, species-grouped row
    return {"aev": atoms + nl + feat * D * N,
            "aev_adjoint": atoms + nl + 4 * Fg * N + 12 * P + 12 * N,   # edge gradients, own-row sums
            "forces": 4 * (N + 1) + 4 * P + 16 * P + 16 * N + 12 * N,   # rev, reverse gradients, own sums, F
            "neighbors": 12 * N + nl + 4 * P}.get(stage, 0)


def source_digest(stage):
    import hashlib
    path = os.path.join(ROOT, "paper_2405_01491_amd", "csrc", STAGE_SOURCE.get(stage, ""))
    if not os.path.isfile(path):
        return None
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def load_traffic(path, stage, config, precision, nets=1):
    """Measured HBM bytes per launch of the stage's kernel (FETCH_SIZE +
    WRITE_SIZE counters scaled by a plain-copy calibration), or None when no
    measurement exists or the kernel source changed since it was taken."""
    path = path or os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.isfile(path):
        return None
    with open(path) as f:
        tab = json.load(f)
    e = tab.get("%s/config%d/%s%s" % (stage, config, precision, "/nets%d" % nets if nets > 1 else ""))
    if not e or e.get("source_sha256") != source_digest(stage):
        return None
    return e


def host_cpu():
    """(model name, logical CPUs available to this process)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return model, n


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        return 1


def oracle_eval(w, spec):
    import oracle
    return oracle.energy_forces(w.pos, w.species, w.mol if w.n_mol > 1 else None, w.n_mol, w.box, spec)


def cpu_baseline(w, spec, single_thread=True):
    """The FP64 oracle (never tuned for speed) on the same workload: one full
    energy + forces evaluation (neighbour search, AEV, networks, adjoint) with
    the host's BLAS threads, and one with a single thread.  Returns the
    record and the oracle's result (the reference for the error table)."""
    cpu_model, ncpu = host_cpu()
    cores = blas_threads()
    t0 = time.perf_counter()
    ref = oracle_eval(w, spec)
    t_all = time.perf_counter() - t0
    rec = {"value": w.n_atoms / t_all, "unit": "atom-steps/s", "cores": int(cores), "kind": "oracle",
           "sample": "one full energy+forces evaluation of the same %d-atom system (cell-binned neighbour search, "
                     "AEV, MLP, adjoint) in %.1f s; numpy float64, BLAS threads = %d (only the network products "
                     "are threaded)" % (w.n_atoms, t_all, cores),
           "cpu_model": cpu_model, "nproc": ncpu}
    if single_thread:
        try:
            from threadpoolctl import threadpool_limits
            with threadpool_limits(limits=1):
                t0 = time.perf_counter()
                oracle_eval(w, spec)
                t_one = time.perf_counter() - t0
            rec["single_thread"] = {"value": w.n_atoms / t_one, "unit": "atom-steps/s", "cores": 1,
                                    "seconds": t_one}
        except ImportError:
            pass
    return rec, ref


def error_row(e_mol, ea, F, ref, spec):
    """Errors of one evaluation against the FP64 oracle: per-atom energy
    relative to max(|E_i|, rms E) and absolute; structure energy relative to
    its magnitude, to the self-energy-free scale sum_i |E_i - e_s| and
    absolute; max and rms force (eV/A)."""
    Er = ref["E_atom"]
    rms = float(np.sqrt(np.mean(Er ** 2)))
    se = np.asarray(spec.self_energy, dtype=np.float64)
    dF = F - ref["F"]
    dE = abs(float(e_mol) - ref["E_mol"][0])
    return {"E_atom_rel": float(np.max(np.abs(ea - Er) / np.maximum(np.abs(Er), rms))),
            "E_atom_max_abs_eV": float(np.max(np.abs(ea - Er))),
            "E_mol_rel": dE / max(abs(ref["E_mol"][0]), 1e-30),
            "E_mol_rel_net_scale": dE / max(float(np.sum(np.abs(Er - se[ref["species"]]))), 1e-30),
            "E_mol_abs_eV": dE,
            "F_max_abs": float(np.abs(dF).max()), "F_rms": float(np.sqrt(np.mean(dF ** 2))),
            "F_ref_rms": float(np.sqrt(np.mean(ref["F"] ** 2)))}


def precision_errors(models, w, ref, spec):
    """Both forms against the FP64 oracle on the workload's starting
    configuration, every atom."""
    import torch
    import paper_2405_01491_amd as nnp
    dev = torch.device("cuda", 0)
    pos = torch.from_numpy(w.pos).to(dev)
    sp = torch.from_numpy(w.species).to(dev)
    ref = dict(ref, species=w.species.astype(np.int64))
    out = {}
    for name, model in models.items():
        nl = nnp.nnp_neighbors(model, pos, None, 1, w.box, model.spec.rc_r)
        e, ea, F = nnp.nnp_energy_forces(model, pos, sp, None, 1, w.box, nl, e_atom=True)
        out[name] = error_row(float(e[0]), ea.cpu().numpy().astype(np.float64),
                              F.cpu().numpy().astype(np.float64), ref, spec)
    return out


def synthetic_masses(w):
    import synthetic
    return synthetic.MASSES[w.species]


def make_engine(model, w, integ, temperature, friction, skin, every, log_every=0, log_capacity=0, dt=0.5,
                seed=2024):
    import torch
    from paper_2405_01491_amd import md as nmd
    dev = torch.device("cuda", 0)
    masses = synthetic_masses(w)
    vel = torch.from_numpy(nmd.maxwell_boltzmann(masses, 300.0, seed=seed)).to(dev)
    return nmd.MDEngine(model, torch.from_numpy(w.pos).to(dev), vel, torch.from_numpy(w.species).to(dev), masses,
                        w.box, dt=dt, integrator=integ, temperature=temperature, friction=friction, seed=seed,
                        skin=skin, rebuild_every=every, log_every=log_every, log_capacity=log_capacity)


def md_form(spec, w, precision, integ, temperature, friction, skin, every, steps, warmup):
    """Atom-steps/s of the same MD workload with another precision form."""
    import torch
    import paper_2405_01491_amd as nnp
    model = nnp.Model(spec, precision)
    sim = make_engine(model, w, integ, temperature, friction, skin, every)
    sim.run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(steps)
    torch.cuda.synchronize()
    dt_s = time.perf_counter() - t0
    info = sim.info()
    sim.close()
    return model, {"value": w.n_atoms * steps / dt_s, "ms_per_step": 1e3 * dt_s / steps,
                   "rebuilds_total": info["rebuilds"], "early_rebuilds": info["early_rebuilds"],
                   "dtype": "f32" if precision == "fp32" else "f32+bf16(mlp)"}


def nve_drift(spec, n_mol=216, dt=0.1, steps=10000, log_every=100):
    """The energy-conservation study of the paper's precision comparison, on a
    short run: NVE velocity Verlet of a 216-water box (648 atoms, 1.0 g/cm^3)
    at dt = 0.1 fs from 300 K, list rebuilt every step, for each precision
    form.  Reports the total energy's largest excursion and its standard
    deviation over the run, in eV and relative to |E_tot(0)| and to the mean
    kinetic energy."""
    import torch
    import synthetic
    import paper_2405_01491_amd as nnp
    w = synthetic.water_box(n_mol, seed=1216)
    out = {"workload": "%d waters (%d atoms), L = %.3f A, NVE dt = %g fs, %d steps (%.1f ps), energy logged every "
                       "%d steps" % (n_mol, w.n_atoms, float(w.box[0]), dt, steps, steps * dt * 1e-3, log_every)}
    for precision in ("fp32", "bf16"):
        model = nnp.Model(spec, precision)
        eng = make_engine(model, w, "nve", 300.0, 0.0, 0.0, 1, log_every=log_every,
                          log_capacity=steps // log_every + 1, dt=dt, seed=1216)
        _, v0, _, ep0 = eng.state()
        m = torch.from_numpy(synthetic_masses(w)).double().to(v0.device)
        from paper_2405_01491_amd import md as nmd
        e_start = float(ep0[0]) + float(0.5 * (m[:, None] * v0.double() ** 2).sum() / nmd.ACC_UNIT)
        t0 = time.perf_counter()
        eng.run(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        rows = eng.log()
        eng.close()
        tot = np.concatenate([[e_start], rows.sum(1)])
        e0 = e_start
        ke = float(rows[:, 1].mean())
        out[precision] = {"E_tot0_eV": float(e0), "max_abs_dev_eV": float(np.abs(tot - e0).max()),
                          "std_eV": float(np.std(tot)), "max_abs_dev_rel_E_tot0": float(np.abs(tot - e0).max() / abs(e0)),
                          "max_abs_dev_rel_KE": float(np.abs(tot - e0).max() / ke), "mean_KE_eV": ke,
                          "drift_eV_per_ps": float(np.polyfit(np.arange(len(tot)) * log_every * dt * 1e-3, tot, 1)[0]),
                          "last_minus_first_eV": float(tot[-1] - e0),
                          "ms_per_step": 1e3 * wall / steps}
    return out


def cluster_latency(spec, reps=200):
    """Latency of one plain-path call on the 72-atom water cluster (24
    waters, open): neighbour list, energy and forces, results on the host."""
    import torch
    import synthetic
    import paper_2405_01491_amd as nnp
    dev = torch.device("cuda", 0)
    w = synthetic.workload(1)
    model = nnp.Model(spec, "fp32")
    pos = torch.from_numpy(w.pos).to(dev)
    sp = torch.from_numpy(w.species).to(dev)
    ts = []
    for k in range(reps + 20):
        t0 = time.perf_counter()
        nl = nnp.nnp_neighbors(model, pos, None, 1, None, spec.rc_r)
        e, _, f = nnp.nnp_energy_forces(model, pos, sp, None, 1, None, nl)
        e.cpu()
        f.cpu()
        if k >= 20:
            ts.append(time.perf_counter() - t0)
    ts = np.array(ts) * 1e3
    return {"workload": "water_cluster_72: 24 waters, open, FP32; nnp_neighbors + nnp_energy_forces + copy to host",
            "p50_ms": float(np.percentile(ts, 50)), "p99_ms": float(np.percentile(ts, 99)), "calls": reps}


def serving_run(model, mols, rate, duration_s, warmup_s, seed, max_inflight=4):
    """Open-loop Poisson stream of single-molecule requests through the
    continuous-batching server; latency = time from the scheduled arrival to
    the moment nnp_poll returns the result."""
    from paper_2405_01491_amd.server import Server, nnp_poll, nnp_submit
    rng = np.random.default_rng(seed)
    pool = len(mols)
    n_req = int((duration_s + warmup_s) * rate)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_req))
    which = rng.integers(0, pool, size=n_req)
    srv = Server(model, arena_bytes=256 << 20, max_slots=8192, max_inflight=max_inflight)
    lat = np.full(n_req, np.nan)
    pending = {}
    k = 0
    done = 0
    t0 = time.perf_counter()
    while done < n_req:
        now = time.perf_counter() - t0
        while k < n_req and arrivals[k] <= now:
            p, s = mols[which[k]]
            t = nnp_submit(srv, s, p)
            if t is None:
                break                      # server full: retry on the next pass (latency keeps counting)
            pending[t] = k
            k += 1
        for t in list(pending):
            r = nnp_poll(srv, t)
            if r is not None:
                j = pending.pop(t)
                lat[j] = time.perf_counter() - t0 - arrivals[j]
                done += 1
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    sel = arrivals >= warmup_s
    L = lat[sel] * 1e3
    atoms = np.array([len(mols[m][1]) for m in which])
    # throughput over the measured window: requests done / time from the first
    # measured arrival to the last completion
    t_first = arrivals[sel][0] if sel.any() else 0.0
    t_last = float(np.nanmax(arrivals[sel] + lat[sel])) if sel.any() else wall
    span = max(t_last - t_first, 1e-9)
    return {"rate_req_s": rate, "p50_ms": float(np.percentile(L, 50)), "p99_ms": float(np.percentile(L, 99)),
            "max_ms": float(np.max(L)), "requests": int(sel.sum()),
            "throughput_req_s": float(sel.sum() / span), "atoms_per_s": float(atoms[sel].sum() / span),
            "launches": st["launches"], "mean_requests_per_launch": st["batched_requests"] / max(1, st["launches"]),
            "wall_s": wall}


def plain_one_at_a_time(model, mols, which):
    """The same requests one at a time on the plain path (closed loop)."""
    import torch
    import paper_2405_01491_amd as nnp
    dev = torch.device("cuda", 0)
    plain = []
    for j in which:
        p, s = mols[j]
        t1 = time.perf_counter()
        pk = torch.from_numpy(p).to(dev)
        sk = torch.from_numpy(s).to(dev)
        nl = nnp.nnp_neighbors(model, pk, None, 1, None, model.spec.rc_r)
        e, _, f = nnp.nnp_energy_forces(model, pk, sk, None, 1, None, nl)
        e.cpu()
        f.cpu()
        plain.append(time.perf_counter() - t1)
    plain = np.array(plain[10:]) * 1e3
    return {"p50_ms": float(np.percentile(plain, 50)), "p99_ms": float(np.percentile(plain, 99)),
            "max_throughput_req_s": float(1e3 / np.mean(plain))}


def serving_bench(model, duration_s=5.0, warmup_s=1.0, rate=2000.0, pool=600, plain_sample=300, seed=1004,
                  sweep=None):
    import synthetic
    rng = np.random.default_rng(seed)
    mols = [synthetic.serving_molecule(rng) for _ in range(pool)]
    main = serving_run(model, mols, rate, duration_s, warmup_s, seed)
    which = np.random.default_rng(seed + 1).integers(0, pool, size=plain_sample)
    main["mean_atoms_per_request"] = float(np.mean([len(mols[j][1]) for j in range(pool)]))
    main["plain_one_at_a_time"] = plain_one_at_a_time(model, mols, which)
    main["workload"] = ("Poisson %.0f req/s, %.0f s after %.0f s warm-up; molecules of 8-150 atoms (log-uniform), "
                        "chain-grown bonded-like geometries (bonds 0.95-1.6 A), H/C/O/N/S/F/Cl mix, open "
                        "boundaries; each request drawn from a pool of %d generated molecules"
                        % (rate, duration_s, warmup_s, pool))
    if sweep:
        main["sweep"] = [serving_run(model, mols, r, duration_s, warmup_s, seed + 7 + k)
                         for k, r in enumerate(sweep)]
    return main


METRIC = "energy+force atom-steps/s at 1 MI355X (FP32 vs BF16-MLP); p50/p99 request latency"


def roofline_of(dom, stages, w, spec, precision, model, nets, n_pairs, traffic_path, config):
    ms_dom, cnt_dom = stages[dom]
    avg_ms = ms_dom / max(cnt_dom, 1)
    N = w.n_atoms
    fwd, adj = mlp_flops_per_atom(spec.widths)
    if dom == "mlp":
        flop, dense_flop, feats = (fwd + adj) * nets * N, (fwd + adj) * nets * N, float(spec.aev_dim)
        if model.fused_mlp:
            flop, dense_flop, feats = mlp_useful_flops(w, spec, precision, nets)
        peak = MI355X_PEAK["bf16_TFLOPs" if precision == "bf16" else "fp32_TFLOPs"]
        achieved = flop / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": None, "stage": "mlp (per-species networks, forward + adjoint)",
                "algorithmic_per_launch": "%.4g FLOP" % flop,
                "dense_equivalent_per_launch": "%.4g FLOP (every feature; the kernel skips feature blocks that "
                                               "are zero for a whole tile)" % dense_flop,
                "active_features_per_atom": round(feats, 1)}
    else:
        Fg = None
        if dom == "aev_adjoint":
            Fg = float(np.mean([active_features(int(m), spec.n_species) for m in species_masks(w, spec)]))
        byt = stage_bytes(dom, N, n_pairs, precision, spec.aev_dim, Fg)
        achieved = byt / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": MI355X_PEAK["hbm_GBs"], "unit": "GB/s",
                "frac": achieved / MI355X_PEAK["hbm_GBs"], "traffic": None, "stage": dom,
                "algorithmic_per_launch": "%.4g B" % byt}
    roof["avg_launch_ms"] = avg_ms
    roof["kernel"] = STAGE_KERNEL.get((dom, model.fused_mlp), dom)
    if dom == "mlp" and nets > 1:
        roof["kernel"] = "k_mlp_fused (per network, to d1) + k_ens_adj1 (first-layer adjoint over networks)"
    tr = load_traffic(traffic_path, dom, config, precision, nets)
    if tr is not None:
        roof["traffic"] = tr["bytes_per_launch"]
        roof["traffic_source"] = tr["profile"]
    return roof


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", type=int, default=5, choices=[2, 3, 4, 5])
    ap.add_argument("--serving-seconds", type=float, default=5.0)
    ap.add_argument("--serving-sweep", default=None,
                    help="comma-separated request rates (req/s) to sweep in the serving form")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"],
                    help="the headline form (the other one runs beside it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the timed MD forms (no serving, cluster latency or NVE drift study)")
    ap.add_argument("--integrator", default="nve", choices=["nve", "langevin"],
                    help="nve: velocity Verlet (the configured workloads); langevin: BAOAB as in the paper's "
                         "benchmarks")
    ap.add_argument("--nets", type=int, default=1,
                    help="networks of the model: 1 (the paper's benchmarks use the first network of ANI-2x) or an "
                         "ensemble of up to 16 on one shared AEV")
    ap.add_argument("--temperature", type=float, default=300.0)
    ap.add_argument("--friction", type=float, default=1.0, help="Langevin friction, 1/ps")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (reference for FETCH_SIZE/WRITE_SIZE counters)")
    ap.add_argument("--traffic", default=None,
                    help="JSON table of measured HBM bytes per launch (default: profiles/hbm_traffic.json)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (the spatial decomposition "
              "over RCCL is a design, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        dev = torch.device("cuda", 0)
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": a.numel() * 4, "launches": 5}))
        return
    import synthetic
    import paper_2405_01491_amd as nnp
    from paper_2405_01491_amd import md as nmd

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    spec = synthetic.ani2x_like_spec() if args.nets == 1 else synthetic.ani2x_like_ensemble(n_nets=args.nets)
    sweep = [float(r) for r in args.serving_sweep.split(",")] if args.serving_sweep else None
    if args.config == 4:
        model = nnp.Model(spec, args.precision)
        sv = serving_bench(model, duration_s=args.serving_seconds, sweep=sweep)
        print(json.dumps({
            "metric": METRIC, "value": sv["atoms_per_s"], "unit": "atom-steps/s", "n_gpus": 1,
            "steps": sv["requests"], "warmup": 0, "ms_per_step": sv["p50_ms"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32" if args.precision == "fp32" else "f32+bf16(mlp)",
            "data": "synthetic", "config": {"workload": sv["workload"]}, "serving": sv}))
        return
    w = synthetic.workload(args.config)
    precision = args.precision
    other = "bf16" if precision == "fp32" else "fp32"
    model = nnp.Model(spec, precision)
    pos = torch.from_numpy(w.pos).to(dev)
    sp = torch.from_numpy(w.species).to(dev)
    integ = args.integrator
    dyn = ("velocity Verlet" if integ == "nve" else
           "BAOAB Langevin %g K, friction %g/ps" % (args.temperature, args.friction))

    if args.config == 3:
        skin, every = 0.0, 1
        nl = nnp.nnp_neighbors(model, pos, None, 1, w.box, spec.rc_r)
        out = {}

        def step():
            nnp.nnp_energy_forces(model, pos, sp, None, 1, w.box, nl, out=out)
        workload = ("organic_box_23000: 23,000 atoms H/C/O/N/S/F/Cl 50/25/12/8/3/1/1 %%, 0.1 atoms/A^3, "
                    "L = 61.27 A, periodic; energy + forces per step (list built once), %s MLP" % precision)
    else:
        if args.config == 2:
            skin, every = 0.0, 1
            workload = ("water_box_4500: 1500 rigid waters, 1.0 g/cm^3, L = 35.54 A, periodic; %s "
                        "dt = 0.5 fs from 300 K, neighbour list rebuilt every step; %s" % (dyn, precision))
        else:
            skin, every = 0.5, 20
            workload = ("water_box_99999: 33,333 rigid waters, 1.0 g/cm^3, L = 99.905 A, periodic; %s "
                        "dt = 0.5 fs from 300 K, 0.5 A skin, rebuild every 20 steps or when the two largest "
                        "displacements exceed the skin; %s MLP" % (dyn, precision))
        sim = make_engine(model, w, integ, args.temperature, args.friction, skin, every)

    # warm-up with every stage timed (the stage breakdown and the choice of the
    # dominant stage), then the timed run with events around that stage only
    nmd.profile_enable(model, True)
    if args.config == 3:
        for _ in range(args.warmup):
            step()
    else:
        sim.run(args.warmup)
    torch.cuda.synchronize()
    warm = nmd.profile_read(model)
    warm_steps = max(args.warmup, 1)
    ranked = {k: ms for k, (ms, cnt) in warm.items() if cnt > 0}
    dom = max(ranked, key=ranked.get) if ranked else "mlp"
    nmd.profile_enable(model, True, stages=[dom])
    if args.config != 3:
        info0 = sim.info()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if args.config == 3:
        for _ in range(args.steps):
            step()
    else:
        sim.run(args.steps)          # enqueued in one go, one synchronisation at the end
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = nmd.profile_read(model)
    nmd.profile_enable(model, False)
    nnp.nnp_check(model)
    if args.config == 3:
        n_pairs = int(nl.c.n_pairs)
    else:
        info = sim.info()
        x_now = sim.state()[0]
        n_pairs = int(nnp.nnp_neighbors(model, x_now, None, 1, w.box, info["r_list"]).c.n_pairs)
        sim.close()
    dt_s = t1 - t0
    N = w.n_atoms
    value = N * args.steps / dt_s
    roof = roofline_of(dom, stages, w, spec, precision, model, args.nets, n_pairs, args.traffic, args.config)
    result = {
        "metric": METRIC, "value": value, "unit": "atom-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt_s / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if precision == "fp32" else "f32+bf16(mlp)", "data": "synthetic",
        "config": {"workload": workload + ("; ensemble of %d networks" % args.nets if args.nets > 1 else ""),
                   "n_atoms": N, "precision": precision, "skin_A": skin, "rebuild_every": every,
                   "list_pairs": n_pairs, "networks": args.nets},
        "stages_ms_per_step_warmup": {k: round(ms / warm_steps, 5) for k, (ms, cnt) in warm.items()},
        "roofline": roof,
    }
    if args.config != 3:
        result["config"]["integrator"] = integ
        result["config"]["rebuilds_in_timed_steps"] = info["rebuilds"] - info0["rebuilds"]
        result["config"]["early_rebuilds_in_timed_steps"] = info["early_rebuilds"] - info0["early_rebuilds"]
    models = {precision: model}
    if args.config != 3:
        om, form = md_form(spec, w, other, integ, args.temperature, args.friction, skin, every, args.steps,
                           args.warmup)
    else:
        om = nnp.Model(spec, other)
        nl2 = nnp.nnp_neighbors(om, pos, None, 1, w.box, spec.rc_r)
        out2 = {}
        for _ in range(args.warmup):
            nnp.nnp_energy_forces(om, pos, sp, None, 1, w.box, nl2, out=out2)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(args.steps):
            nnp.nnp_energy_forces(om, pos, sp, None, 1, w.box, nl2, out=out2)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - ta) / args.steps
        form = {"value": N / tb, "ms_per_step": 1e3 * tb, "dtype": "f32" if other == "fp32" else "f32+bf16(mlp)"}
    result["forms"] = {precision: {"value": value, "ms_per_step": result["ms_per_step"], "dtype": result["dtype"]},
                       other: form}
    models[other] = om
    if not args.no_extras and args.config in (2, 5):
        if args.serving_seconds > 0:
            result["serving"] = serving_bench(nnp.Model(spec, "fp32"), duration_s=args.serving_seconds, sweep=sweep)
        result["latency_cluster_72"] = cluster_latency(spec)
        result["nve_drift"] = nve_drift(spec)
    if not args.no_cpu_baseline:
        result["cpu_baseline"], ref = cpu_baseline(w, spec)
        result["precision_vs_fp64_oracle"] = precision_errors(models, w, ref, spec)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
