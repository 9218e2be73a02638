"""Benchmark of the contrastive-RL update on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one whole critic update: relabel + gather from the GPU-resident
replay buffer, phi/psi encoders, critic matrix + InfoNCE + logsumexp penalty,
backward through everything, Adam.  The default workload is the B=4096,
4x1024 LayerNorm+Swish, dot-energy, symmetric-InfoNCE update with BF16 MFMA
tiles and the fused (never materialised) logits; its K steps are replayed
from captured HIP graphs.  Beside it:
  - the same update on the plain FP32 path (FP32 MFMA tiles, materialised
    B x B logits), eager and from a graph;
  - per-kernel times from HIP events in an instrumented eager pass;
  - the full update (the same critic step, then the 4x1024 tanh-Gaussian
    policy step and the entropy-coefficient step), 1000 consecutive steps
    from captured graphs;
  - the B=16384, D=256 L2-energy update (fused: its B x B logits are never
    stored) with its peak HBM use;
  - training iterations on a ring replay buffer: append a freshly unrolled
    chunk of every environment's steps, then a given number of updates (the
    update-to-data ratio), each iteration one captured graph;
  - the FP64 oracle on the host cores, on a bounded sample.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("CRL update steps/s and MFMA TFLOP/s at B=4096, BF16-fused vs plain FP32")
PEAK_BF16_TFLOPS = 2500.0   # MI355X dense BF16 MFMA
PEAK_FP32_TFLOPS = 157.3    # MI355X FP32 matrix
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="b4096_lnswish4x1024_dot_sym")
    ap.add_argument("--graph-steps", type=int, default=10,
                    help="consecutive updates captured in one HIP graph")
    ap.add_argument("--fp32-steps", type=int, default=20)
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--full-workload", default="b4096_full_update_actor4x1024")
    ap.add_argument("--full-steps", type=int, default=1000,
                    help="consecutive full updates (critic, policy, alpha) timed")
    ap.add_argument("--full-graph-steps", type=int, default=1000)
    ap.add_argument("--no-full", action="store_true")
    ap.add_argument("--large-workload", default="b16384_lnswish2x1024_d256_l2_sym")
    ap.add_argument("--large-steps", type=int, default=100,
                    help="updates timed on the large-batch fused workload (never materialises "
                         "the B x B logits)")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--others", default="b256_relu2x256_l2_sym,b1024_lnswish4x1024_l2_fwd",
                    help="further workloads timed from graphs ('' = none)")
    ap.add_argument("--no-rates", action="store_true")
    ap.add_argument("--no-single-thread", action="store_true")
    ap.add_argument("--utd", default="1,16",
                    help="updates per appended chunk timed on the ring buffer ('' = none)")
    ap.add_argument("--utd-iterations", type=int, default=24)
    ap.add_argument("--ring-capacity", type=int, default=1000)
    ap.add_argument("--unroll", type=int, default=62, help="steps per env per append")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="N",
                    help="only run crl_cast_bf16 over N floats 10 times (reads 4N, writes "
                         "2N bytes per launch): the known-size kernel that scales the HBM "
                         "byte counters of a profiler run, then exit")
    return ap.parse_args()


def time_steps(upd, steps, warmup, graph_steps):
    import torch
    for _ in range(warmup):
        upd.enqueue()
    torch.cuda.synchronize()
    if graph_steps > 0:
        g = upd.capture(graph_steps)
        reps = max(1, steps // graph_steps)
        g.replay()  # one untimed replay
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            g.replay()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dt, reps * graph_steps
    t0 = time.perf_counter()
    for _ in range(steps):
        upd.enqueue()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, steps


def kernel_table(upd, steps):
    """Per-kernel HIP-event times over `steps` eager updates."""
    import torch
    from paper_2408_11052_amd import crl_timing_enable, crl_timing_read, crl_timing_reset
    crl_timing_reset()
    crl_timing_enable(True)
    for _ in range(steps):
        upd.enqueue()
    torch.cuda.synchronize()
    crl_timing_enable(False)
    rows = crl_timing_read()
    crl_timing_reset()
    return rows


def host_description():
    """CPU model and the BLAS behind numpy (threadpoolctl's view)."""
    from threadpoolctl import threadpool_info
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = [f"{d.get('internal_api')} {d.get('version')} ({d.get('threading_layer', '?')} "
            f"threads, {d.get('num_threads')} threads)"
            for d in threadpool_info() if d.get("user_api") == "blas"]
    return {"cpu_model": model, "blas": blas, "os_cpu_count": os.cpu_count()}


def oracle_single_thread(w, obs, act, phi, psi):
    """One FP64 oracle update with the BLAS limited to one thread (seconds)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import critic as ocritic
    from oracle import relabel as orelabel
    phi = [{k: a.astype(np.float64) for k, a in L.items()} for L in phi]
    psi = [{k: a.astype(np.float64) for k, a in L.items()} for L in psi]
    with threadpool_limits(limits=1, user_api="blas"):
        t0 = time.perf_counter()
        _, x_sa, x_g, _ = orelabel.sample_relabel(obs, act, w.batch_size, w.discounting, 2, 0,
                                                  w.goal_lo, w.goal_dim)
        ocritic.critic_loss_and_grads(phi, psi, x_sa, x_g, w)
        return time.perf_counter() - t0


def cpu_baseline(w, obs, act, phi, psi, budget_s):
    """The FP64 oracle's update on the host cores, on a bounded sample."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle import adam as oadam
    from oracle import critic as ocritic
    from oracle import relabel as orelabel
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    flat_p = [(k, L) for layers in (phi, psi) for L in layers for k in L]
    m = [np.zeros(L[k].shape) for k, L in flat_p]
    v = [np.zeros(L[k].shape) for k, L in flat_p]
    phi = [{k: a.astype(np.float64) for k, a in L.items()} for L in phi]
    psi = [{k: a.astype(np.float64) for k, a in L.items()} for L in psi]
    steps, t0 = 0, time.perf_counter()
    while True:
        _, x_sa, x_g, _ = orelabel.sample_relabel(obs, act, w.batch_size, w.discounting, 2,
                                                  steps, w.goal_lo, w.goal_dim)
        out = ocritic.critic_loss_and_grads(phi, psi, x_sa, x_g, w)
        i = 0
        for side, layers in (("phi", phi), ("psi", psi)):
            for l, L in enumerate(layers):
                for k in L:
                    L[k], m[i], v[i] = oadam.adam_step(L[k], out["g_" + side][l][k], m[i], v[i],
                                                       steps + 1, w.critic_lr)
                    i += 1
        steps += 1
        dt = time.perf_counter() - t0
        if dt >= budget_s or steps >= 50:
            break
    return {"value": steps / dt, "unit": "update-steps/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{steps} full FP64 updates (relabel, critic fwd+bwd, Adam) of the "
                      f"same workload in {dt:.1f} s"}


def other_workloads(names, dev, steps=100):
    """Updates/s of further workloads (their own buffers), from graphs of 10."""
    import torch
    from paper_2408_11052_amd.update import CriticUpdate, critic_step_flops
    from synthetic import WORKLOADS, buffer_for, critic_params_for
    out = []
    for name in names:
        wo = WORKLOADS[name]
        obs, act = buffer_for(wo, seed=0)
        p, q = critic_params_for(wo, seed=1)
        d_obs, d_act = torch.from_numpy(obs).to(dev), torch.from_numpy(act).to(dev)
        u = CriticUpdate(wo, d_obs, d_act, p, q, seed=2, keep_grads=False)
        dt, n = time_steps(u, steps, 5, 10)
        fl = critic_step_flops(wo)["total"]
        peak = PEAK_BF16_TFLOPS if wo.precision == "bf16" else PEAK_FP32_TFLOPS
        out.append({"workload": name, "precision": wo.precision, "logits": wo.logits,
                    "steps_per_s": round(n / dt, 2), "ms_per_step": round(1e3 * dt / n, 4),
                    "tflops": round(fl * n / dt / 1e12, 3),
                    "frac_of_peak": round(fl * n / dt / 1e12 / peak, 4)})
        log(f"[bench] {name}: {n / dt:.1f} steps/s ({wo.precision})")
        u.close()
        del u, d_obs, d_act
        torch.cuda.empty_cache()
    return out


def training_iterations(w, phi, psi, args, dev):
    """Iterations of (append U steps of every env to the ring, then k updates)
    on a ring of the headline workload's buffer size.  A pool of P chunks
    (one continuous synthetic unroll, time-major) is resident in HBM; graph p
    appends chunk p, so replaying the P graphs in turn cycles through the
    pool.  The ring is filled to capacity before timing."""
    import torch
    from paper_2408_11052_amd import ReplayRing, crl_timing_enable, crl_timing_read, \
        crl_timing_reset
    from paper_2408_11052_amd.update import CriticUpdate, critic_step_flops
    from synthetic.trajectories import unroll_stream
    E, C, U, P = w.num_envs, args.ring_capacity, args.unroll, 4
    log(f"[utd] ring {E} envs x {C} steps, chunks of {U} steps (pool of {P})")
    t0 = time.perf_counter()
    obs, act, traj = unroll_stream(E, P * U, w.obs_dim, w.act_dim, w.episode_len, seed=11)
    pool = [(torch.from_numpy(obs[p * U:(p + 1) * U]).to(dev),
             torch.from_numpy(act[p * U:(p + 1) * U]).to(dev),
             torch.from_numpy(traj[p * U:(p + 1) * U]).to(dev)) for p in range(P)]
    del obs, act, traj
    log(f"[utd] chunk pool ready in {time.perf_counter() - t0:.1f} s")
    ring = ReplayRing(E, C, w.obs_dim, w.act_dim, device=dev)
    for i in range((C + U - 1) // U):
        ring.insert(*pool[i % P])
    torch.cuda.synchronize()
    # the append alone, HIP-event timed
    crl_timing_reset()
    crl_timing_enable(True)
    for i in range(P):
        ring.insert(*pool[i])
    torch.cuda.synchronize()
    crl_timing_enable(False)
    ins = [r for r in crl_timing_read() if r[0] == "replay_insert_kernel"]
    crl_timing_reset()
    out = {"workload": w.name, "num_envs": E, "ring_capacity": C, "unroll": U}
    if ins:
        _, la, kms, _, kby = ins[0]
        out["insert_us"] = round(1e3 * kms / la, 2)
        out["insert_gbs"] = round(kby / (kms * 1e-3) / 1e9, 1)
        out["insert_mb"] = round(kby / la / 1e6, 1)
    fl = critic_step_flops(w)["total"]
    runs = []
    for k in [int(x) for x in args.utd.split(",") if x]:
        upd = CriticUpdate(w, ring, None, phi, psi, seed=2, keep_grads=False)
        graphs = [upd.capture_iteration(*pool[p], updates=k) for p in range(P)]
        for g in graphs:  # untimed
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.utd_iterations):
            graphs[i % P].replay()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        its = args.utd_iterations / dt
        runs.append({"updates_per_append": k, "iterations_per_s": round(its, 2),
                     "updates_per_s": round(its * k, 2),
                     "env_steps_per_s": round(its * E * U, 1),
                     "ms_per_iteration": round(1e3 * dt / args.utd_iterations, 4),
                     "tflops": round(fl * k * its / 1e12, 2),
                     "loss": round(float(upd.loss[0]), 5)})
        log(f"[utd] {k} updates per append: {its:.1f} iterations/s, {its * k:.1f} updates/s")
        del graphs
        upd.close()
        del upd
        torch.cuda.empty_cache()
    out["runs"] = runs
    del ring, pool
    torch.cuda.empty_cache()
    return out


def source_digest(files) -> str:
    """sha256 (first 16 hex digits) over library source files, in the given order."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2408_11052_amd", "csrc")
    for f in files:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/hbm_traffic_b4096.txt: FETCH_SIZE and WRITE_SIZE per dispatch,
    scaled by the copy calibration), or None if it holds no line for this
    kernel or the sources that define the kernel changed since the counters
    were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_b4096.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if not line.startswith("kernel "):
            continue
        parts = dict(p.split("=", 1) for p in line.split()[1:])
        if parts.get("name") != kernel:
            continue
        try:
            if source_digest(parts["sources"].split(",")) != parts["sha"]:
                return None
        except (KeyError, OSError):
            return None
        return float(parts["hbm_bytes_per_launch"])
    return None


def copy_calibration(n):
    import torch
    from paper_2408_11052_amd import crl_cast_bf16
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty(n, dtype=torch.bfloat16, device="cuda:0")
    torch.cuda.synchronize()
    for _ in range(10):
        crl_cast_bf16(src, dst)
    torch.cuda.synchronize()
    log(f"[calibration] crl_cast_bf16 over {n} floats x10: reads {4 * n} B, writes {2 * n} B "
        f"per launch")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(this build runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2408_11052_amd import lib
    from paper_2408_11052_amd.update import CriticUpdate, critic_step_flops, adam_bytes
    from synthetic import WORKLOADS, buffer_for, critic_params_for

    lib()  # fail loudly if the library is not built
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    w = WORKLOADS[args.workload]
    log(f"[bench] workload {w.name}: generating the replay buffer "
        f"({w.num_envs} x {w.episode_len} x {w.obs_dim})")
    t0 = time.perf_counter()
    obs, act = buffer_for(w, seed=0)
    phi, psi = critic_params_for(w, seed=1)
    log(f"[bench] buffer ready in {time.perf_counter() - t0:.1f} s; uploading")
    dev = torch.device("cuda:0")
    d_obs = torch.from_numpy(obs).to(dev)
    d_act = torch.from_numpy(act).to(dev)
    torch.cuda.synchronize()

    flops = critic_step_flops(w)
    upd = CriticUpdate(w, d_obs, d_act, phi, psi, seed=2, keep_grads=False)
    nparam = upd.crit.nparam
    ws_gib = upd.crit.ws_bytes / 2**30
    log(f"[bench] {w.precision}/{w.logits}: {upd.crit.nparam} params, workspace "
        f"{upd.crit.ws_bytes / 2**20:.1f} MiB; timing {args.steps} steps "
        f"(graphs of {args.graph_steps})")
    dt, n = time_steps(upd, args.steps, args.warmup, args.graph_steps)
    ms = 1e3 * dt / n
    sps = n / dt
    tflops = flops["total"] * sps / 1e12
    loss = upd.loss.cpu().numpy().tolist()
    log(f"[bench] {sps:.1f} steps/s, {ms:.3f} ms/step, {tflops:.1f} TFLOP/s algorithmic; "
        f"loss parts after {int(upd.n.item())} steps: {[round(x, 4) for x in loss[:4]]}")
    peak_mem = torch.cuda.max_memory_allocated() / 2**30

    roofline, kernels = None, []
    if not args.no_profile:
        rows = kernel_table(upd, args.profile_steps)
        tot = sum(r[2] for r in rows) or 1.0
        for name, la, kms, kfl, kby in sorted(rows, key=lambda r: -r[2]):
            kernels.append({"kernel": name, "launches": la, "ms_total": round(kms, 4),
                            "us_avg": round(1e3 * kms / max(la, 1), 2),
                            "share": round(kms / tot, 4),
                            "tflops": round(kfl / (kms * 1e-3) / 1e12, 2) if kfl else None,
                            "gbs": round(kby / (kms * 1e-3) / 1e9, 1) if kby else None})
            log(f"[kernels] {name:34s} n={la:4d} avg {1e3 * kms / max(la, 1):9.2f} us "
                f"share {kms / tot:6.1%} "
                + (f"{kfl / (kms * 1e-3) / 1e12:8.1f} TFLOP/s " if kfl else "")
                + (f"{kby / (kms * 1e-3) / 1e9:8.1f} GB/s" if kby else ""))
        top = max(rows, key=lambda r: r[2])
        name, la, kms, kfl, kby = top
        if kfl > 0:
            # operand precision: the direct-to-LDS GEMM and the fused InfoNCE
            # kernels always multiply BF16; gemm_kernel names its storage type first
            bf16_in = (name.startswith("gemm_lds_") or name.startswith("gemm_kernel<bf16")
                       or name.startswith("infonce"))
            peak = PEAK_BF16_TFLOPS if bf16_in else PEAK_FP32_TFLOPS
            ach = kfl / la / (kms * 1e-3 / la) / 1e12
            roofline = {"bound": "mfma", "kernel": name, "achieved": round(ach, 2),
                        "peak": peak, "unit": "TFLOP/s", "frac": round(ach / peak, 4),
                        "flops_per_launch": kfl / la, "us_per_launch": 1e3 * kms / la,
                        "traffic": measured_traffic(name)}
        else:
            ach = kby / la / (kms * 1e-3 / la) / 1e9
            roofline = {"bound": "hbm", "kernel": name, "achieved": round(ach, 1),
                        "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4),
                        "bytes_per_launch": kby / la, "us_per_launch": 1e3 * kms / la,
                        "traffic": measured_traffic(name)}
    upd.close()
    del upd
    torch.cuda.empty_cache()

    fp32 = None
    if not args.no_fp32:
        wf = w.with_(precision="fp32", logits="materialised")
        upf = CriticUpdate(wf, d_obs, d_act, phi, psi, seed=2, keep_grads=False)
        log(f"[bench] plain FP32 path (materialised logits, eager): {args.fp32_steps} steps")
        dtf, nf = time_steps(upf, args.fp32_steps, 2, 0)
        dtg, ng = time_steps(upf, args.fp32_steps, 0, 5)
        fp32 = {"steps_per_s": round(nf / dtf, 2), "ms_per_step": round(1e3 * dtf / nf, 3),
                "graph_steps_per_s": round(ng / dtg, 2),
                "tflops": round(flops["total"] * nf / dtf / 1e12, 2)}
        log(f"[bench] FP32 plain: {nf / dtf:.1f} steps/s eager, {ng / dtg:.1f} steps/s graph")
        upf.close()
        del upf
        torch.cuda.empty_cache()

    full = None
    if not args.no_full:
        from paper_2408_11052_amd.update import FullUpdate, actor_step_flops
        from synthetic import actor_params
        wa = WORKLOADS[args.full_workload]
        assert (wa.num_envs, wa.episode_len, wa.obs_dim, wa.act_dim) == \
            (w.num_envs, w.episode_len, w.obs_dim, w.act_dim), "full update needs the same buffer"
        pa, qa = critic_params_for(wa, seed=1)
        actor = actor_params(wa.in_sg, wa.actor_hidden, wa.act_dim,
                             wa.activation == "ln_swish", seed=3)
        fu = FullUpdate(wa, d_obs, d_act, pa, qa, actor, seed=2, keep_grads=False)
        fl = critic_step_flops(wa)["total"] + actor_step_flops(wa)["total"]
        log(f"[bench] full update {wa.name}: {fu.crit.nparam_actor} policy params; "
            f"{args.full_steps} steps from graphs of {args.full_graph_steps}")
        dfu, nfu = time_steps(fu, args.full_steps, 2, args.full_graph_steps)
        full = {"workload": wa.name, "steps": nfu, "graph_steps": args.full_graph_steps,
                "steps_per_s": round(nfu / dfu, 2), "ms_per_step": round(1e3 * dfu / nfu, 4),
                "gflop_per_step": round(fl / 1e9, 3),
                "tflops": round(fl * nfu / dfu / 1e12, 2),
                "critic_loss": round(float(fu.loss[0]), 5),
                "actor_loss": round(float(fu.actor_loss[0]), 5),
                "log_alpha": round(float(fu.log_alpha[0]), 5)}
        log(f"[bench] full update: {nfu / dfu:.1f} steps/s, {1e3 * dfu / nfu:.3f} ms/step, "
            f"{fl * nfu / dfu / 1e12:.1f} TFLOP/s; after {int(fu.n.item())} steps critic "
            f"{full['critic_loss']}, actor {full['actor_loss']}, log alpha {full['log_alpha']}")
        fu.close()
        del fu
        torch.cuda.empty_cache()

    large = None
    if not args.no_large:
        wl = WORKLOADS[args.large_workload]
        log(f"[bench] large-batch workload {wl.name}: buffer {wl.num_envs} x {wl.episode_len} x "
            f"{wl.obs_dim}")
        lobs, lact = buffer_for(wl, seed=0)
        lp, lq = critic_params_for(wl, seed=1)
        ld_obs = torch.from_numpy(lobs).to(dev)
        ld_act = torch.from_numpy(lact).to(dev)
        del lobs, lact
        torch.cuda.reset_peak_memory_stats()
        lu = CriticUpdate(wl, ld_obs, ld_act, lp, lq, seed=2, keep_grads=False)
        lfl = critic_step_flops(wl)["total"]
        dtl, nl = time_steps(lu, args.large_steps, 5, 10)
        peak_l = torch.cuda.max_memory_allocated() / 2**30
        # the B x B FP32 logits this workload never stores
        dense = wl.batch_size * wl.batch_size * 4 / 2**30
        large = {"workload": wl.name, "batch": wl.batch_size, "steps": nl,
                 "steps_per_s": round(nl / dtl, 2), "ms_per_step": round(1e3 * dtl / nl, 4),
                 "gflop_per_step": round(lfl / 1e9, 3),
                 "tflops": round(lfl * nl / dtl / 1e12, 2),
                 "tflops_frac_bf16_peak": round(lfl * nl / dtl / 1e12 / PEAK_BF16_TFLOPS, 4),
                 "peak_hbm_gib": round(peak_l, 2), "workspace_gib": round(lu.crit.ws_bytes / 2**30, 3),
                 "dense_logits_gib_not_stored": round(dense, 2),
                 "loss": round(float(lu.loss[0]), 5)}
        log(f"[bench] large batch: {nl / dtl:.1f} steps/s, {1e3 * dtl / nl:.3f} ms/step, "
            f"{lfl * nl / dtl / 1e12:.1f} TFLOP/s; peak HBM {peak_l:.2f} GiB (buffer included), "
            f"workspace {lu.crit.ws_bytes / 2**30:.2f} GiB; B x B logits would be {dense:.2f} GiB")
        lu.close()
        del lu, ld_obs, ld_act
        torch.cuda.empty_cache()

    utd = None
    if args.utd:
        utd = training_iterations(w, phi, psi, args, dev)

    others = None
    if args.others:
        others = other_workloads(args.others.split(","), dev)

    rates = None
    if not args.no_rates:
        from paper_2408_11052_amd import crl_peak_rate
        exp_rate = crl_peak_rate("exp")
        fma_rate = crl_peak_rate("fma32")
        rates = {"exp_per_s": exp_rate, "fma32_per_s": fma_rate,
                 "fp32_vector_tflops_unpacked": round(2 * fma_rate / 1e12, 2)}
        # the D = 64 InfoNCE kernels: two exponentials per critic-matrix entry
        # (row and column log-sum-exp in the forward; P^r and P^c in the
        # backward), so the exponential issue rate bounds them
        exps = 2.0 * w.batch_size * w.batch_size
        rk = []
        for k in kernels:
            if k["kernel"].startswith("infonce_"):
                per = k["us_avg"] * 1e-6
                rk.append({"kernel": k["kernel"], "exps_per_launch": exps,
                           "us_per_launch": k["us_avg"],
                           "achieved_exp_per_s": exps / per,
                           "frac_of_exp_rate": round(exps / per / exp_rate, 4)})
        rates["exp_bound_kernels"] = rk
        log(f"[bench] measured rates: {exp_rate / 1e12:.2f} T exp/s, {fma_rate / 1e12:.2f} T "
            f"FP32 FMA/s; " + ", ".join(f"{r['kernel']} {r['frac_of_exp_rate']:.1%} of the exp "
                                         f"rate" for r in rk))

    cpu = None
    if not args.no_cpu:
        log(f"[bench] FP64 oracle on the host cores (~{args.cpu_seconds:.0f} s)")
        cpu = cpu_baseline(w, obs, act, phi, psi, args.cpu_seconds)
        log(f"[bench] oracle: {cpu['value']:.3f} steps/s on {cpu['cores']} threads")
        cpu["host"] = host_description()
        if not args.no_single_thread:
            st = oracle_single_thread(w, obs, act, phi, psi)
            cpu["single_thread_steps_per_s"] = round(1.0 / st, 4)
            log(f"[bench] oracle, one BLAS thread: {st:.1f} s per update")

    out = {
        "metric": METRIC,
        "value": round(sps, 2),
        "unit": "update-steps/s",
        "n_gpus": 1,
        "steps": n,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if w.precision == "bf16" else "fp32",
        "data": "synthetic",
        "config": {"workload": w.name, "batch": w.batch_size, "obs_dim": w.obs_dim,
                   "act_dim": w.act_dim, "goal_dim": w.goal_dim,
                   "hidden": list(w.hidden), "repr_dim": w.repr_dim,
                   "activation": w.activation, "energy": w.energy_function,
                   "loss": w.contrastive_loss_function, "logits": w.logits,
                   "buffer": [w.num_envs, w.episode_len], "graph_steps": args.graph_steps,
                   "parallelism": "single GPU"},
        "tflops": round(tflops, 2),
        "tflops_frac_bf16_peak": round(tflops / PEAK_BF16_TFLOPS, 4),
        "gflop_per_step": round(flops["total"] / 1e9, 3),
        "adam_bytes_per_step": adam_bytes(nparam, w.precision == "bf16"),
        "fp32_plain": fp32,
        "speedup_vs_fp32_plain": round(sps / fp32["steps_per_s"], 2) if fp32 else None,
        "peak_hbm_gib": round(peak_mem, 2),
        "workspace_gib": round(ws_gib, 3),
        "full_update": full,
        "large_batch": large,
        "training_iterations": utd,
        "other_workloads": others,
        "issue_rates": rates,
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
