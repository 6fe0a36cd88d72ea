"""Train-step throughput of the NEP loss-and-gradient path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: 512 periodic Sb-Te-shaped structures with atom counts log-uniform in
32-512 (about 88k atoms; rocksalt-like, liquid-like and amorphous cells,
density 0.029-0.033 /A^3), NEP with 3/4/5-body terms (n_rad 7, n_ang 5,
basis 11, l 4/2/1, hidden 50), teacher labels plus noise.  One step =
neighbor lists, energies/forces/virials, loss, parameter gradient and Adam.

  batched: the whole step captured once as a HIP graph and replayed;
  plain:   a host loop over structures, one neighbor build and one
           loss-and-gradient call per structure through the same C ABI,
           gradients summed with the batch's global normalisation, then Adam.

Prints one JSON line.  Inputs are resident in HBM before timing starts.  The
same run also times the batched step on the 27,000-atom cell and on the
2,000-structure set (`workloads`), and the FP64 oracle on the host's cores
(`cpu_baseline`).
"""
from __future__ import annotations

import argparse
import ctypes as C
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "train-step atoms/s (E+F+virial+param grad), batched vs plain, 1 MI355X"
PEAK_FP32_VECTOR = 157.3e12   # MI355X fp32 vector (packed FP32), FLOP/s
PEAK_FP32_NONPACKED = 78.6e12  # one FP32 FMA per lane per clock: 256 CUs x 4 SIMDs x 16 lanes x 2 x 2.4 GHz
PEAK_HBM = 8.0e12             # bytes/s
MAX_CPU_WORKERS = 15          # oracle worker processes (each opens the GPU device through torch)


# --------------------------------------------------------------- FLOP model
def flop_model(sz, mR: float, mA: float) -> dict:
    """Algorithmic FLOPs per atom of each heavy kernel (an FMA counts 2), with
    mR, mA the mean radial/angular neighbors per atom.  Each term is the
    arithmetic the mathematics needs once; recomputation inside a kernel is
    not counted."""
    T, NR, NA, KR, KA, H, D = sz.n_types, sz.n_rad, sz.n_ang, sz.k_rad, sz.k_ang, sz.hidden, sz.n_desc
    lmax = max(min(sz.l3, 4), sz.l4, sz.l5)   # harmonics of the per-atom kernels
    Y = lmax * (lmax + 2)
    YH = (sz.l3 + 1) ** 2 - 25 if sz.l3 > 4 else 0   # l = 5..l3, in kernels of their own
    geo = 13                       # d = x_j + sL - x_i, r^2, sqrt, 1/r
    tan = 20                       # t = Fbar_j - Fbar_i + Gamma d, r_hat . t
    basis = lambda K: 10 + 6 * K        # xi, cutoff, T_k recursion, f_k
    basis_d = lambda K: 14 + 17 * K     # ... plus T'_k recursion and f'_k
    harm = 2 * Y                   # b_lm(u), l <= 4
    harm_grad = 3 * Y              # grad b_lm(u)
    q4 = 60 if sz.l4 else 0
    q5 = 8 if sz.l5 else 0
    fwd = (mR * (geo + basis(KR) + KR)                                   # radial sums F_Jk
           + 2 * T * NR * KR                                             # q_n
           + mA * (geo + basis(KA) + 2 * NA * KA + harm + 2 * NA * Y)    # g_n, S_nlm
           + NA * (3 * Y + q4 + q5)                                      # q_nl, q4, q5
           + 4 * H * D + 12 * H                                          # network, E'
           + 2 * T * NR * KR + NA * (3 * Y + q4 + q5)                    # h_Jk, A_nlm
           + mR * (geo + basis_d(KR) + 2 * KR + 15)                      # radial partial forces, virial
           + mA * (geo + basis_d(KA) + 4 * NA * KA + harm + harm_grad
                   + 4 * NA * Y + 8 * Y + 27))                           # angular partial forces, virial
    adj = (mR * (geo + tan + basis_d(KR) + 4 * KR)                       # F_Jk, Fp_Jk
           + 2 * T * NR * KR                                             # radial Gdot
           + mA * (geo + tan + basis_d(KA) + 4 * NA * KA + harm + harm_grad
                   + 7 * Y + 4 * NA * Y)                                 # Sdot
           + NA * (4 * Y + 2 * q4 + q5)                                  # angular Gdot
           + 4 * H * D + 14 * H                                          # a, beta, Gbar, NN partials
           + 4 * T * NR * KR                                             # radial coefficient gradient
           + NA * (8 * Y + 4 * q4 + 2 * q5)                              # Sbar, A
           + mA * (6 * NA * Y + 4 * NA * KA))                            # X_n, Y_n, angular coefficient gradient
    outer = 4 * H * D + 4 * NR * T * KR   # dW0 and dc^R, contracted over atoms (one launch)
    out = {"forward": fwd, "adjoint": adj, "outer_sums_reduce": outer}
    if YH:
        hv, hg = 2 * YH, 3 * YH    # harmonic values and gradients of l = 5..l3
        out["high_desc"] = mA * (geo + basis(KA) + 2 * NA * KA + hv + 2 * NA * YH) + 2 * NA * YH
        out["high_force"] = (2 * NA * YH + mA * (geo + basis_d(KA) + 4 * NA * KA + hv + hg
                                                 + 4 * NA * YH + 6 * YH + 27))
        out["high_tangent"] = mA * (geo + tan + basis_d(KA) + 4 * NA * KA + hv + hg + 6 * YH
                                    + 4 * NA * YH) + 3 * NA * YH
        out["high_coef"] = 5 * NA * YH + mA * (geo + tan + basis_d(KA) + hv + hg + 6 * YH + 6 * NA * YH
                                               + 4 * NA * KA)
    return out


def step_flops_formula(sz, mR: float, mA: float) -> float:
    """Whole-step FLOPs per atom by the closed formula of the hot-path scope
    (basis recomputed in the forward, force and adjoint passes):
    radial m_R (18 K_R + 60 + 10 n_R K_R), angular m_A (18 K_A + 60 + 101 Y
    + 9 n_A K_A + 16 n_A Y), network 12 D H."""
    lmax = max(sz.l3, sz.l4, sz.l5)
    Y = lmax * (lmax + 2)
    rad = mR * (18 * sz.k_rad + 60 + 10 * sz.n_rad * sz.k_rad)
    ang = mA * (18 * sz.k_ang + 60 + 101 * Y + 9 * sz.n_ang * sz.k_ang + 16 * sz.n_ang * Y)
    return rad + ang + 12 * sz.n_desc * sz.hidden


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("paper_2507_00528_amd/csrc/nep_lib.hip", "paper_2507_00528_amd/csrc/nep_device.h",
              "paper_2507_00528_amd/csrc/nep_kernels.h", "paper_2507_00528_amd/csrc/nep_highl.h"):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, only if
    it was taken on the current kernel sources."""
    p = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def measured_counters(kernel: str, workload: str):
    """SQ busy fractions of a kernel from the committed rocprofv3 counter
    summary, only if it was taken on the current kernel sources."""
    p = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("source_hash") != kernel_source_hash():
        return None
    return {k: d[k] for k in ("valu_busy", "mfma_busy", "valu_instr_per_wave") if k in d}


# ------------------------------------------------------- CPU baseline (oracle)
_W = {}


def _cpu_worker_init(sizes, theta, lam):
    import torch
    torch.set_num_threads(1)
    from oracle import NEPOracle
    _W.update(o=NEPOracle(sizes), theta=theta, lam=lam)


def _cpu_worker(task):
    """One structure's neighbor lists, loss and gradient on the FP64 oracle."""
    st, lab = task
    o = _W["o"]
    nb = o.neighbors(st)
    L, g = o.loss_and_grad(_W["theta"], [st], lab, _W["lam"], nbr_cache=[nb])
    return st.n, g


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sizes, structures, theta_np, e_lab, f_lab, w_lab, lam, budget_s, log):
    """The FP64 oracle (neighbors, loss and gradient of every structure of the
    batch) over a process pool of one worker per host core, each worker one
    torch thread; the median of up to three full passes.

    Every worker imports torch, and on a ROCm host that opens the GPU device
    even though the oracle runs on the CPU.  A GPU host allows at most 16
    processes with the device open, this one included, so the pool takes at
    most MAX_CPU_WORKERS of the cores."""
    import multiprocessing as mp
    cores = min(len(os.sched_getaffinity(0)), MAX_CPU_WORKERS)
    offs = np.cumsum([0] + [st.n for st in structures])
    tasks = []
    for k, st in enumerate(structures):
        lab = dict(energy=e_lab[k:k + 1].astype(np.float64),
                   force=[f_lab[:, offs[k]:offs[k + 1]].T.astype(np.float64)],
                   virial=w_lab[k:k + 1].astype(np.float64))
        tasks.append((st, lab))
    order = sorted(range(len(tasks)), key=lambda k: -structures[k].n)   # largest first: balanced tail
    tasks = [tasks[k] for k in order]
    walls = []
    with mp.get_context("spawn").Pool(cores, initializer=_cpu_worker_init, initargs=(sizes, theta_np, lam)) as pool:
        pool.map(_cpu_worker, tasks[-cores:], chunksize=1)   # every worker has imported and built its oracle
        t_all = time.perf_counter()
        while len(walls) < 3:
            t0 = time.perf_counter()
            atoms = 0
            grad = np.zeros(len(theta_np))
            for n, g in pool.imap_unordered(_cpu_worker, tasks, chunksize=1):
                atoms += n
                grad += g
            walls.append(time.perf_counter() - t0)
            if time.perf_counter() - t_all > budget_s:
                break
    wall = float(np.median(walls))
    log(f"cpu oracle: {atoms / wall:.1f} atoms/s on {cores} worker processes ({len(walls)} passes)")
    return {"value": atoms / wall, "unit": "atoms/s", "cores": cores, "host_cores": len(os.sched_getaffinity(0)),
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"the whole batch: {len(structures)} structures, {atoms} atoms; neighbors, loss and "
                      f"gradient in FP64 (torch CPU), one structure per task over {cores} processes of one "
                      f"thread each; median wall time of {len(walls)} passes ({wall:.2f}s)"}


# ---------------------------------------------------------------- the bench
WORKLOAD_TEXT = {
    "c2": "512 structures, atom counts log-uniform in 32-512 (rocksalt-like, liquid, amorphous)",
    "c3": "one amorphous Sb2Te3-stoichiometry cell of 27,000 atoms (RSA, min distance 2.7 A)",
    "c4": "2,000 structures of 32-1,024 atoms, p(N) ~ 1/N^2 (adds 10% hot liquid)",
}


def _generate(name):
    from paper_2507_00528_amd import synth
    return synth.config_structures(name)


class Workload:
    """Device state of one workload: batch, lists, teacher labels plus noise."""

    def __init__(self, name, sizes, structures, log):
        import torch
        from paper_2507_00528_amd import nep, synth
        self.name, self.sizes, self.structures = name, sizes, structures
        self.batch = synth.Batch(structures)
        self.S, self.N = self.batch.n_struct, self.batch.n_atom
        self.model = nep.Model.of(sizes)
        self.P = nep.param_count(self.model)
        self.dev = nep.DeviceBatch(self.batch)
        self.nbrs = nep.Neighbors(self.model, self.N)
        self.ws = nep.workspace(self.model, self.S, self.N)
        self.flags = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.theta = torch.tensor(synth.draw_params(self.P, synth.SEEDS["student"]), device="cuda")
        self.teacher = torch.tensor(synth.draw_params(self.P, synth.SEEDS["teacher"]), device="cuda")
        nep.build_neighbors(self.model, self.dev, self.nbrs, self.ws, self.flags)
        e_t = torch.zeros(self.S, device="cuda")
        f_t = torch.zeros(3 * self.N, device="cuda")
        w_t = torch.zeros(6 * self.S, device="cuda")
        nep.energy_force_virial(self.model, self.dev, self.nbrs, self.teacher, self.ws, None, e_t, f_t, w_t)
        de, df = synth.label_noise(self.batch, synth.SEEDS["noise"])
        self.labels = nep.Labels(e_t + torch.tensor(de, dtype=torch.float32, device="cuda"),
                                 f_t + torch.tensor(df, dtype=torch.float32, device="cuda"), w_t)
        torch.cuda.synchronize()
        nep.check_flags(self.flags, f"{name} neighbors")
        self.cnt_r = self.nbrs.cnt_rad.float().mean().item()
        self.cnt_a = self.nbrs.cnt_ang.float().mean().item()
        log(f"workload {name}: {self.S} structures, {self.N} atoms, mean neighbors {self.cnt_r:.2f} / "
            f"{self.cnt_a:.2f}")

    def batched(self, steps, warmup, lam, lr, stream, log, cached=False, persistent=False, tuning="cache"):
        """The captured train step replayed `steps` times after `warmup`
        replays; one event between consecutive replays.  persistent: the step
        after the neighbor build as one persistent launch; tuning: launch
        choices (None: the library defaults, "cache": the autotuner's)."""
        import torch
        from paper_2507_00528_amd import nep
        nb, ws, fl = self.nbrs, self.ws, self.flags
        if cached:
            nb = nep.Neighbors(self.model, self.N)
            ws = nep.workspace(self.model, self.S, self.N)
            fl = torch.zeros(1, dtype=torch.int32, device="cuda")
            nep.build_neighbors(self.model, self.dev, nb, ws, fl)
        params = self.theta.clone()
        m, v, grad = (torch.zeros(self.P, device="cuda") for _ in range(3))
        loss = torch.zeros(4, device="cuda")
        step = torch.ones(1, dtype=torch.int32, device="cuda")
        graph = nep.TrainStepGraph(self.model, self.dev, nb, self.labels, lam, params, m, v, grad, loss, step, ws,
                                   fl, lr_start=lr, lr_stop=lr, stream=stream, cached_neighbors=cached,
                                   persistent=persistent, tuning=tuning)
        self.last_tuning = dict(graph.tuning)
        torch.cuda.synchronize()   # inputs were filled on the default stream
        with torch.cuda.stream(stream):
            for _ in range(warmup):
                graph.launch(stream)
        stream.synchronize()
        loss_first = loss.cpu().numpy().copy()
        nep.check_flags(fl, f"{self.name} graph warmup")
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        evs[0].record(stream)
        for k in range(steps):
            graph.launch(stream)
            evs[k + 1].record(stream)
        stream.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        ms = evs[0].elapsed_time(evs[-1]) / steps
        per = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(steps)])
        loss_last = loss.cpu().numpy().copy()
        nep.check_flags(fl, f"{self.name} graph replays")
        graph.close()
        dist = {"median_ms": float(np.median(per)), "p10_ms": float(np.percentile(per, 10)),
                "p90_ms": float(np.percentile(per, 90))}
        log(f"{self.name} {'cached' if cached else 'batched'}{' persistent' if persistent else ''} "
            f"{graph.tuning or 'defaults'}: "
            f"{ms:.3f} ms/step (events), "
            f"{1e3 * wall / steps:.3f} ms/step (wall), median {dist['median_ms']:.3f}; "
            f"loss {loss_first[0]:.5g} -> {loss_last[0]:.5g}")
        return ms, dist, (loss_first, loss_last)

    def both_paths(self, steps, warmup, lam, lr, stream, log):
        """The forms of the captured step: separate launches with the library's
        hand-set launch choices, with the autotuner's cached choices (when it
        has some for this size class), and the persistent form."""
        from paper_2507_00528_amd import nep, tune
        out = {"graph": self.batched(steps, warmup, lam, lr, stream, log, tuning=None)}
        choices = tune.lookup(self.model, self.dev)
        self.tuned_choices = choices
        if choices:
            out["graph_tuned"] = self.batched(steps, warmup, lam, lr, stream, log, tuning=choices)
        if not (choices or {}).get("persistent"):
            try:
                out["persistent"] = self.batched(steps, warmup, lam, lr, stream, log, persistent=True, tuning=None)
            except nep.NEPError as e:   # a batch or model the persistent step does not cover
                log(f"{self.name}: no persistent step ({e})")
        return out

    def kernels(self, reps, lam, stream):
        """Mean per-kernel times (HIP events on the launch stream) of the
        unfused loss-and-gradient launches."""
        import torch
        from paper_2507_00528_amd import nep
        prof = {}
        g2 = torch.zeros(self.P, device="cuda")
        l2 = torch.zeros(4, device="cuda")
        for _ in range(reps):
            for name, ms in nep.profile_loss_grad(self.model, self.dev, self.nbrs, self.theta, self.labels, lam, l2,
                                                  g2, self.ws, self.flags, stream=stream):
                prof.setdefault(name, []).append(ms)
        return {k: float(np.mean(v)) for k, v in prof.items()}

    def roofline(self, kern_ms, ms_step, profile_name):
        fm = flop_model(self.sizes, self.cnt_r, self.cnt_a)
        dom = max(kern_ms, key=kern_ms.get)
        flops = fm.get(dom, 0.0) * self.N
        achieved = flops / (kern_ms[dom] * 1e-3)
        traffic = measured_traffic(dom, profile_name) if profile_name else None
        counters = measured_counters(dom, profile_name) if profile_name else None
        step_fpa = step_flops_formula(self.sizes, self.cnt_r, self.cnt_a)
        step_rate = step_fpa * self.N / (ms_step * 1e-3)
        return {"bound": "alu", "kernel": dom, "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR, "traffic": traffic,
                "flops_per_atom": fm.get(dom, 0.0), "units": self.N, "kernel_ms": kern_ms[dom],
                "frac_of_nonpacked_peak": achieved / PEAK_FP32_NONPACKED,
                "hbm_frac": (traffic / (kern_ms[dom] * 1e-3) / PEAK_HBM) if traffic else None,
                "counters": counters,
                "step": {"flops_per_atom_formula": step_fpa,
                         "flops_per_atom_kernels": float(sum(fm.values())),
                         "achieved": step_rate / 1e12, "frac": step_rate / PEAK_FP32_VECTOR,
                         "frac_of_nonpacked_peak": step_rate / PEAK_FP32_NONPACKED}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--profile-reps", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=25.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--skip-plain", action="store_true")
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--extra", default="c3,c4",
                    help="further workloads measured in the same run (batched step and roofline), '' for none")
    ap.add_argument("--extra-steps", type=int, default=20)
    ap.add_argument("--sizes", default=None, choices=[None, "large", "small", "l8"],
                    help="model sizes in place of the workload's own (l8: 3-body degrees up to 8)")
    ap.add_argument("--mode", default="full", choices=["full", "batched", "copy-probe"],
                    help="full: the JSON line; batched: graph replays only (for profilers); "
                         "copy-probe: a plain 512 MiB device copy, the HBM-counter calibration")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the data-parallel sharding of "
              "structures across GPUs is not part of this build.", file=sys.stderr)
        sys.exit(2)

    def log(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    # the extra workloads' structures are drawn in the background while the
    # main workload runs (geometry only: seeded RSA and lattices)
    extra = [w for w in args.extra.split(",") if w and w != args.workload] if args.mode == "full" else []
    gen = None
    if extra:
        import concurrent.futures as cf
        import multiprocessing as mp
        gen = cf.ProcessPoolExecutor(max_workers=len(extra), mp_context=mp.get_context("spawn"))
        futs = {w: gen.submit(_generate, w) for w in extra}

    import torch
    from paper_2507_00528_amd import nep, synth

    if args.mode == "copy-probe":
        n = 512 * 1024 * 1024 // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: 3 copies of {4 * n} bytes")
        return

    t0 = time.time()
    sizes = (synth.CONFIG_SIZES[args.workload] if args.sizes is None else
             {"large": synth.SIZES_LARGE, "small": synth.SIZES_SMALL, "l8": synth.SIZES_L8}[args.sizes])
    structures = synth.config_structures(args.workload)
    log(f"workload {args.workload} generated in {time.time() - t0:.1f}s")
    W = Workload(args.workload, sizes, structures, log)
    S, N, P, model = W.S, W.N, W.P, W.model
    lam = (1.0, 1.0, 0.1)
    lr = 1e-3
    stream = torch.cuda.Stream()

    # reference loss and gradient at the initial parameters (eager calls)
    loss0 = torch.zeros(4, device="cuda")
    grad0 = torch.zeros(P, device="cuda")
    nep.loss_grad(model, W.dev, W.nbrs, W.theta, W.labels, lam, loss0, grad0, W.ws, W.flags)
    torch.cuda.synchronize()
    loss0 = loss0.cpu().numpy()
    grad0 = grad0.cpu().numpy()

    # the two forms of the captured step: separate launches, and the step after
    # the neighbor build as one persistent launch; the faster one is the value
    paths = W.both_paths(args.steps, args.warmup, lam, lr, stream, log)
    best = min(paths, key=lambda k: paths[k][0])
    ms_batched, dist, (loss_first, loss_last) = paths[best]
    # context only: the same step with the lists built once beforehand
    ms_cached, _, _ = W.batched(args.steps, args.warmup, lam, lr, stream, log, cached=True)
    if args.mode == "batched":
        return

    # ---------------- plain: per-structure launches through the same ABI
    plain_out = None
    if not args.skip_plain:
        lib = nep._lib.load()
        offs = W.batch.atom_offset
        nmax = int(np.diff(offs).max())
        ws_p = nep.workspace(model, 1, nmax)
        nb_p = nep.Neighbors(model, nmax)
        nb_c = nb_p.c()
        mc = model.c()
        e_lab = W.labels.energy.cpu().numpy()
        f_lab = W.labels.force.cpu().numpy().reshape(3, N)
        w_lab = W.labels.virial.cpu().numpy().reshape(S, 6)
        per = []
        for k, st in enumerate(structures):
            db = nep.DeviceBatch(synth.Batch([st]))
            a0, a1 = offs[k], offs[k + 1]
            lb = nep.Labels(torch.tensor(e_lab[k:k + 1], device="cuda"),
                            torch.tensor(np.ascontiguousarray(f_lab[:, a0:a1]).reshape(-1), device="cuda"),
                            torch.tensor(w_lab[k], device="cuda"))
            lam_k = (C.c_float * 3)(lam[0] / S, lam[1] * st.n / N, lam[2] / S)
            per.append((db, db.c(), lb, lb.c(), lam_k))
        params_p = W.theta.clone()
        m_p = torch.zeros(P, device="cuda")
        v_p = torch.zeros(P, device="cuda")
        grad_p = torch.zeros(P, device="cuda")
        gacc = torch.zeros(P, device="cuda")
        lacc = torch.zeros(4, device="cuda")
        loss_p = torch.zeros(4, device="cuda")
        sp = C.c_void_p(stream.cuda_stream)
        ptr = lambda t: C.c_void_p(t.data_ptr())

        def plain_step(it):
            gacc.zero_()
            lacc.zero_()
            for db, dbc, lb, lbc, lam_k in per:
                rc = lib.nep_build_neighbors(C.byref(mc), C.byref(dbc), C.byref(nb_c), ptr(ws_p), ptr(W.flags), sp)
                rc |= lib.nep_loss_grad(C.byref(mc), C.byref(dbc), C.byref(nb_c), ptr(params_p), C.byref(lbc),
                                        C.byref(lam_k), ptr(loss_p), ptr(grad_p), None, None, None, ptr(ws_p),
                                        ptr(W.flags), sp)
                if rc:
                    raise RuntimeError(f"plain step failed: {rc}")
                gacc.add_(grad_p)
                lacc.add_(loss_p)
            nep.adam_step(params_p, m_p, v_p, gacc, lr, it, stream=stream)

        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            plain_step(1)
            stream.synchronize()
            loss_plain_first = float(lacc[0].item())
            gdiff = float(np.abs(gacc.cpu().numpy() - grad0).max() / max(np.abs(grad0).max(), 1e-30))
            torch.cuda.synchronize()
            tp = time.perf_counter()
            for it in range(2, 2 + args.plain_steps):
                plain_step(it)
            stream.synchronize()
            ms_plain = 1e3 * (time.perf_counter() - tp) / args.plain_steps
        log(f"plain: {ms_plain:.2f} ms/step; loss at theta {loss_plain_first:.6g} vs batched {loss0[0]:.6g}; "
            f"gradient max rel diff {gdiff:.2e}")
        plain_out = {"value": N / (ms_plain * 1e-3), "unit": "atoms/s", "ms_per_step": ms_plain,
                     "speedup_batched_over_plain": ms_plain / ms_batched,
                     "loss_at_theta": loss_plain_first, "grad_max_rel_diff_vs_batched": gdiff}

    # ---------------- per-kernel timing (HIP events on the launch stream)
    kern_ms = W.kernels(args.profile_reps, lam, stream)
    roof = W.roofline(kern_ms, ms_batched, args.workload if args.sizes is None else None)
    log("kernels (ms): " + ", ".join(f"{k} {v:.4f}" for k, v in sorted(kern_ms.items(), key=lambda x: -x[1])))

    # ---------------- the other workloads: batched step and roofline
    others = {}
    for w in extra:
        t1 = time.time()
        sts = futs[w].result()
        log(f"workload {w} ready after {time.time() - t1:.1f}s of waiting")
        Wx = Workload(w, synth.CONFIG_SIZES[w], sts, log)
        px = Wx.both_paths(args.extra_steps, 3, lam, lr, stream, log)
        bx = min(px, key=lambda k: px[k][0])
        msx, distx, _ = px[bx]
        msx_c, _, _ = Wx.batched(args.extra_steps, 3, lam, lr, stream, log, cached=True)
        kx = Wx.kernels(2, lam, stream)
        others[w] = {"workload": WORKLOAD_TEXT.get(w, w), "structures": Wx.S, "atoms": Wx.N,
                     "ms_per_step": msx, "value": Wx.N / (msx * 1e-3), "unit": "atoms/s", "path": bx,
                     "tuned_choices": Wx.tuned_choices,
                     "step_paths_ms": {k: v[0] for k, v in px.items()},
                     "replay_distribution": distx,
                     "cached_neighbors": {"ms_per_step": msx_c, "value": Wx.N / (msx_c * 1e-3)},
                     "mean_neighbors_rad": Wx.cnt_r, "mean_neighbors_ang": Wx.cnt_a,
                     "roofline": Wx.roofline(kx, msx, w), "kernels_ms": kx}
        del Wx
        torch.cuda.empty_cache()
    if gen is not None:
        gen.shutdown()

    # ---------------- CPU baseline: the FP64 oracle over the host's cores
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(sizes, structures, W.theta.cpu().numpy(), W.labels.energy.cpu().numpy(),
                           W.labels.force.cpu().numpy().reshape(3, N), W.labels.virial.cpu().numpy().reshape(S, 6),
                           lam, args.cpu_seconds, log)

    value = N / (ms_batched * 1e-3)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "atoms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_batched,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: seeded RSA/rocksalt Sb-Te-shaped cells, teacher-NEP labels plus noise",
        "config": {"workload": f"{args.workload}: {S} structures, {N} atoms, "
                               f"{WORKLOAD_TEXT.get(args.workload, '')}; "
                               f"NEP n_rad {sizes.n_rad} n_ang {sizes.n_ang} basis {sizes.k_rad} "
                               f"l {sizes.l3}/{sizes.l4}/{sizes.l5} hidden {sizes.hidden}",
                   "structures": S, "atoms": N, "mean_neighbors_rad": W.cnt_r, "mean_neighbors_ang": W.cnt_a,
                   "path": f"batched HIP-graph train step (neighbors+E/F/W+loss+grad+Adam), {best} form"},
        "step_paths": {k: {"ms_per_step": v[0], "value": N / (v[0] * 1e-3), "replay_distribution": v[1]}
                       for k, v in paths.items()},
        "tuning": {"cached_choices": W.tuned_choices,
                   "note": "graph: the library's hand-set launch choices; graph_tuned: the autotuner's cached "
                           "choices for this size class (paper_2507_00528_amd/tune.py)"},
        "plain": plain_out,
        "roofline": roof,
        "replay_distribution": dist,
        "cached_neighbors": {"ms_per_step": ms_cached, "value": N / (ms_cached * 1e-3), "unit": "atoms/s",
                             "note": "context only: lists built once before timing"},
        "kernels_ms": kern_ms,
        "workloads": others,
        "cpu_baseline": cpu,
        "loss": {"at_theta": float(loss0[0]), "after_warmup": float(loss_first[0]),
                 "after_steps": float(loss_last[0])},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
