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

Prints one JSON line.  Inputs are resident in HBM before timing starts.
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
PEAK_FP32_VECTOR = 157.3e12   # MI355X fp32 vector, FLOP/s
PEAK_HBM = 8.0e12             # bytes/s


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
    out = {"forward": fwd, "adjoint": adj, "outer_sums": outer}
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


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("paper_2507_00528_amd/csrc/nep_lib.hip", "paper_2507_00528_amd/csrc/nep_device.h",
              "paper_2507_00528_amd/csrc/nep_kernels.h"):
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


# ---------------------------------------------------------------- the bench
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--profile-reps", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--skip-plain", action="store_true")
    ap.add_argument("--workload", default="c2")
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

    import torch
    from paper_2507_00528_amd import nep, synth

    def log(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

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
    batch = synth.Batch(structures)
    S, N = batch.n_struct, batch.n_atom
    log(f"workload {args.workload}: {S} structures, {N} atoms, generated in {time.time() - t0:.1f}s")
    model = nep.Model.of(sizes)
    P = nep.param_count(model)
    dev = nep.DeviceBatch(batch)
    nbrs = nep.Neighbors(model, N)
    ws = nep.workspace(model, S, N)
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    theta = torch.tensor(synth.draw_params(P, synth.SEEDS["student"]), device="cuda")
    teacher = torch.tensor(synth.draw_params(P, synth.SEEDS["teacher"]), device="cuda")

    # teacher labels (GPU forward) plus seeded noise
    nep.build_neighbors(model, dev, nbrs, ws, flags)
    e_t = torch.zeros(S, device="cuda")
    f_t = torch.zeros(3 * N, device="cuda")
    w_t = torch.zeros(6 * S, device="cuda")
    nep.energy_force_virial(model, dev, nbrs, teacher, ws, None, e_t, f_t, w_t)
    de, df = synth.label_noise(batch, synth.SEEDS["noise"])
    labels = nep.Labels(e_t + torch.tensor(de, dtype=torch.float32, device="cuda"),
                        f_t + torch.tensor(df, dtype=torch.float32, device="cuda"), w_t)
    torch.cuda.synchronize()
    nep.check_flags(flags, "neighbors")
    cnt_r = nbrs.cnt_rad.float().mean().item()
    cnt_a = nbrs.cnt_ang.float().mean().item()
    lam = (1.0, 1.0, 0.1)
    lr = 1e-3
    stream = torch.cuda.Stream()

    # reference loss and gradient at the initial parameters (eager calls)
    loss0 = torch.zeros(4, device="cuda")
    grad0 = torch.zeros(P, device="cuda")
    nep.loss_grad(model, dev, nbrs, theta, labels, lam, loss0, grad0, ws, flags)
    torch.cuda.synchronize()
    loss0 = loss0.cpu().numpy()
    grad0 = grad0.cpu().numpy()

    # ---------------- batched: captured train step
    params = theta.clone()
    m = torch.zeros(P, device="cuda")
    v = torch.zeros(P, device="cuda")
    grad = torch.zeros(P, device="cuda")
    loss = torch.zeros(4, device="cuda")
    step = torch.ones(1, dtype=torch.int32, device="cuda")
    graph = nep.TrainStepGraph(model, dev, nbrs, labels, lam, params, m, v, grad, loss, step, ws, flags,
                               lr_start=lr, lr_stop=lr, stream=stream)
    torch.cuda.synchronize()   # inputs were filled on the default stream
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            graph.launch(stream)
    stream.synchronize()
    loss_first = loss.cpu().numpy().copy()
    nep.check_flags(flags, "graph warmup")
    # one event between consecutive replays: the total gives ms_per_step, the
    # differences the per-replay distribution
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    evs[0].record(stream)
    for k in range(args.steps):
        graph.launch(stream)
        evs[k + 1].record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_batched = evs[0].elapsed_time(evs[-1]) / args.steps
    per_replay = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)])
    dist = {"median_ms": float(np.median(per_replay)), "p10_ms": float(np.percentile(per_replay, 10)),
            "p90_ms": float(np.percentile(per_replay, 90))}
    loss_last = loss.cpu().numpy().copy()
    nep.check_flags(flags, "graph replays")
    log(f"batched: {ms_batched:.3f} ms/step (events), {1e3 * wall / args.steps:.3f} ms/step (wall), "
        f"median {dist['median_ms']:.3f} p10 {dist['p10_ms']:.3f} p90 {dist['p90_ms']:.3f}; "
        f"loss {loss_first[0]:.5g} -> {loss_last[0]:.5g}")

    # context only: the same step with the neighbor lists built once beforehand
    # (training positions never change); the metric above rebuilds them
    nb_c = nep.Neighbors(model, N)
    ws_c = nep.workspace(model, S, N)
    fl_c = torch.zeros(1, dtype=torch.int32, device="cuda")
    nep.build_neighbors(model, dev, nb_c, ws_c, fl_c)
    pc = theta.clone()
    mc_, vc_, gc_ = (torch.zeros(P, device="cuda") for _ in range(3))
    lc_ = torch.zeros(4, device="cuda")
    sc_ = torch.ones(1, dtype=torch.int32, device="cuda")
    graph_c = nep.TrainStepGraph(model, dev, nb_c, labels, lam, pc, mc_, vc_, gc_, lc_, sc_, ws_c, fl_c,
                                 lr_start=lr, lr_stop=lr, stream=stream, cached_neighbors=True)
    torch.cuda.synchronize()   # lists and buffers come from the default stream; the replays run on `stream`
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            graph_c.launch(stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        graph_c.launch(stream)
    e1.record(stream)
    stream.synchronize()
    nep.check_flags(fl_c, "cached-neighbor replays")
    ms_cached = e0.elapsed_time(e1) / args.steps
    graph_c.close()
    log(f"cached neighbors: {ms_cached:.3f} ms/step")
    if args.mode == "batched":
        return

    # ---------------- plain: per-structure launches through the same ABI
    plain_out = None
    if not args.skip_plain:
        lib = nep._lib.load()
        offs = batch.atom_offset
        nmax = int(np.diff(offs).max())
        ws_p = nep.workspace(model, 1, nmax)
        nb_p = nep.Neighbors(model, nmax)
        nb_c = nb_p.c()
        mc = model.c()
        e_lab = labels.energy.cpu().numpy()
        f_lab = labels.force.cpu().numpy().reshape(3, N)
        w_lab = labels.virial.cpu().numpy().reshape(S, 6)
        per = []
        for k, st in enumerate(structures):
            db = nep.DeviceBatch(synth.Batch([st]))
            a0, a1 = offs[k], offs[k + 1]
            lb = nep.Labels(torch.tensor(e_lab[k:k + 1], device="cuda"),
                            torch.tensor(np.ascontiguousarray(f_lab[:, a0:a1]).reshape(-1), device="cuda"),
                            torch.tensor(w_lab[k], device="cuda"))
            lam_k = (C.c_float * 3)(lam[0] / S, lam[1] * st.n / N, lam[2] / S)
            per.append((db, db.c(), lb, lb.c(), lam_k))
        params_p = theta.clone()
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
                rc = lib.nep_build_neighbors(C.byref(mc), C.byref(dbc), C.byref(nb_c), ptr(ws_p), ptr(flags), sp)
                rc |= lib.nep_loss_grad(C.byref(mc), C.byref(dbc), C.byref(nb_c), ptr(params_p), C.byref(lbc),
                                        C.byref(lam_k), ptr(loss_p), ptr(grad_p), None, None, None, ptr(ws_p),
                                        ptr(flags), sp)
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
    prof = {}
    g2 = torch.zeros(P, device="cuda")
    l2 = torch.zeros(4, device="cuda")
    for _ in range(args.profile_reps):
        for name, ms in nep.profile_loss_grad(model, dev, nbrs, theta, labels, lam, l2, g2, ws, flags,
                                              stream=stream):
            prof.setdefault(name, []).append(ms)
    kern_ms = {k: float(np.mean(v)) for k, v in prof.items()}
    dom = max(kern_ms, key=kern_ms.get)
    fm = flop_model(sizes, cnt_r, cnt_a)
    units = N
    flops = fm.get(dom, 0.0) * units
    achieved = flops / (kern_ms[dom] * 1e-3)
    traffic = measured_traffic(dom, args.workload) if args.sizes is None else None
    counters = measured_counters(dom, args.workload) if args.sizes is None else None
    log("kernels (ms): " + ", ".join(f"{k} {v:.4f}" for k, v in sorted(kern_ms.items(), key=lambda x: -x[1])))

    # ---------------- CPU baseline: the FP64 oracle on a bounded sample
    cpu = None
    if not args.no_cpu:
        from oracle import NEPOracle
        o = NEPOracle(sizes)
        th_np = theta.cpu().numpy()
        tt_np = teacher.cpu().numpy()
        done_atoms, spent, k = 0, 0.0, 0
        while spent < args.cpu_seconds and k < S:
            st = structures[k]
            nb = o.neighbors(st)
            pt = o.predict(tt_np, [st], [nb])
            lab = dict(energy=pt["E"], force=pt["F"], virial=pt["W"])
            tc = time.perf_counter()
            o.loss_and_grad(th_np, [st], lab, lam, nbr_cache=[nb])
            spent += time.perf_counter() - tc
            done_atoms += st.n
            k += 1
        cpu = {"value": done_atoms / spent, "unit": "atoms/s", "cores": int(torch.get_num_threads()),
               "kind": "oracle",
               "sample": f"first {k} of {S} structures ({done_atoms} atoms), FP64 torch loss and gradient, "
                         f"{spent:.1f}s"}
        log(f"cpu oracle: {cpu['value']:.1f} atoms/s on {cpu['cores']} threads")

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
        "config": {"workload": f"{args.workload}: {S} structures, {N} atoms, sizes log-uniform 32-512, "
                               f"NEP n_rad {sizes.n_rad} n_ang {sizes.n_ang} basis {sizes.k_rad} "
                               f"l {sizes.l3}/{sizes.l4}/{sizes.l5} hidden {sizes.hidden}",
                   "structures": S, "atoms": N, "mean_neighbors_rad": cnt_r, "mean_neighbors_ang": cnt_a,
                   "path": "batched HIP-graph train step (neighbors+E/F/W+loss+grad+Adam)"},
        "plain": plain_out,
        "roofline": {"bound": "alu", "kernel": dom, "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR, "traffic": traffic,
                     "flops_per_atom": fm.get(dom, 0.0), "units": units, "kernel_ms": kern_ms[dom],
                     "frac_of_nonpacked_peak": achieved / (PEAK_FP32_VECTOR / 2),
                     "hbm_frac": (traffic / (kern_ms[dom] * 1e-3) / PEAK_HBM) if traffic else None,
                     "counters": counters},
        "replay_distribution": dist,
        "cached_neighbors": {"ms_per_step": ms_cached, "value": N / (ms_cached * 1e-3), "unit": "atoms/s",
                             "note": "context only: lists built once before timing"},
        "kernels_ms": kern_ms,
        "cpu_baseline": cpu,
        "loss": {"at_theta": float(loss0[0]), "after_warmup": float(loss_first[0]),
                 "after_steps": float(loss_last[0])},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
