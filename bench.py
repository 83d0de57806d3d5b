"""Throughput of the forward model + hand-written adjoint (logL gradient
evaluations per second) on one MI355X, with the roofline of the dominant kernel
class and the FP64 CPU oracle timed beside it.

Workload (default): 256^3 mesh, L = 1000 Mpc/h, Phi-web (R=8) x delta-web (R=2),
16 regions, plane-parallel RSD along z, mean count 2, NB dispersion 3; seeded
synthetic white noise and synthetic counts.  One step = one forward + adjoint
(value_and_grad) of that chain.  Also reported: the same step with 4 identical
256^3 chains batched in one plan (grads/s counts every chain).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--copy-calibration]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, 8 TB/s

# kernel of each timing class with the four-step FFT schedule (rocprofv3 names)
KERNEL_SYMBOLS = {
    "z_r2c": "fzw::zpass4_r2c_kernel<{n}>", "z_c2r": "fzw::zpass4_c2r_kernel<{n}>",
    "y_mix": "fzw::xy4_pass_kernel<{n}, 1, 1, false>", "x_mix": "fzw::xy4_pass_kernel<{n}, 0, 1, false>",
    "y_mix_multi": "fzw::xy4_pass_kernel<{n}, 1, 1, true>", "x_mix_multi": "fzw::xy4_pass_kernel<{n}, 0, 1, true>",
    "y_pure": "fzw::xy4_pure_kernel<{n}, 1, *>", "x_pure": "fzw::xy4_pure_kernel<{n}, 0, *>",
    "lpt_fwd": "fzw::lpt_fwd_z4_kernel<{n}>", "lpt_bwd": "fzw::lpt_bwd_z4_kernel<{n}>",
    "cic_adjoint": "fzw::cic_adjoint_kernel", "voxel_fwd": "fzw::voxel_fwd_kernel<{w}>",
    "likelihood": "fzw::likelihood_kernel", "voxel_bwd": "fzw::voxel_bwd_kernel<{w}>"}


# sources whose kernels the stored byte counters describe
TRAFFIC_SOURCES = ("paper_2506_03969_amd/csrc/fzw_fft.hip", "paper_2506_03969_amd/csrc/fzw_device.hpp",
                   "paper_2506_03969_amd/csrc/fzw_internal.hpp")


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel_class, n):
    """HBM bytes per launch of a kernel class from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy), or
    None when there is none or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%d.json" % (kernel_class, n))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_sha256") != sources_sha256():
        return None
    return float(d["hbm_bytes_per_launch"])


# every library source: the whole-gradient traffic figure describes all kernels
ALL_SOURCES = ("paper_2506_03969_amd/csrc/fzw_fft.hip", "paper_2506_03969_amd/csrc/fzw_ops.hip",
               "paper_2506_03969_amd/csrc/fzw_nuts.hip", "paper_2506_03969_amd/csrc/fzw_stats.hip",
               "paper_2506_03969_amd/csrc/fzw_plan.cpp", "paper_2506_03969_amd/csrc/fzw_device.hpp",
               "paper_2506_03969_amd/csrc/fzw_internal.hpp", "paper_2506_03969_amd/csrc/fzw_ops.hpp")


def all_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel in ALL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_gradient_traffic(n):
    """HBM bytes of one whole forward+adjoint (every kernel's FETCH_SIZE and
    WRITE_SIZE, scaled by a plain copy) from the committed rocprofv3 summary,
    or None when there is none or any library source changed since."""
    path = os.path.join(ROOT, "profiles", "traffic_gradient_%d.json" % n)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_sha256") != all_sources_sha256():
        return None
    return float(d["hbm_bytes_per_gradient"])


def gradients_only(k, workload, torch):
    """Plan creation and k forward+adjoint evaluations, nothing else: the
    command the whole-gradient byte counters are collected on."""
    import numpy as np
    import fzw_inputs as fi
    from paper_2506_03969_amd import CosmoParams, Plan, WebParams
    w = fi.workload(workload)
    ch = w.chains[0]
    plan = _plan(w, [ch], Plan, CosmoParams, WebParams)
    plan.set_counts(0, torch.from_numpy(fi.timing_counts(ch).view(np.int16)).cuda())
    nu = torch.from_numpy(fi.white_noise(ch, fi.ROLE_EVAL_NU).astype(np.float32).ravel()).cuda()
    bias = torch.from_numpy(ch.bias.astype(np.float32)[None]).cuda()
    out = (torch.empty(1, dtype=torch.float64, device="cuda"), torch.empty_like(nu), torch.empty_like(bias))
    for _ in range(k):
        plan.value_and_grad(nu, bias, out)
    torch.cuda.synchronize()
    print(json.dumps({"gradients_only": k, "workload": workload}), flush=True)


def _plan(w, chains, Plan, CosmoParams, WebParams, checkpoint=False):
    c = w.cosmo
    cosmo = CosmoParams(c.omega_m, c.h, c.sigma8, c.n_s, c.d1, c.f_growth, c.r_s, c.rsd_axis, c.tau_sc,
                        c.x_floor)
    web = WebParams(w.web.kinds, w.web.smooth_r, w.web.ell, w.web.steepness, w.web.lambda_th)
    return Plan([ch.n for ch in chains], [ch.box for ch in chains], cosmo, web, checkpoint=checkpoint)


def _time_steps(plan, nu, bias, out, steps, torch):
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(plan.stream)
    for _ in range(steps):
        plan.value_and_grad(nu, bias, out)
    ev1.record(plan.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return ev0.elapsed_time(ev1) / 1e3, wall


def cpu_baseline(w, n_cpu=128, reps=3):
    """The FP64 oracle (as it stands) on a bounded sample of the same model:
    forward + adjoint at n_cpu^3 with the same cell size, one untimed warm-up
    then the median of `reps` runs, reported as the rate at that mesh (not
    scaled to another size).  Threads: the host's share (OMP_NUM_THREADS when
    set) for the FFTs; the batched 3x3 eigen-solver and the element-wise
    NumPy work run on one thread."""
    import statistics
    import fzw_inputs as fi
    from oracle import model as om
    ncpu = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count() or 1
    om.set_workers(ncpu)
    ws = fi.small_variant(w, n_cpu)
    ch = ws.chains[0]
    m = om.Model(om.Settings.from_workload(ws.cosmo, ws.web, ch))
    nu = fi.white_noise(ch, fi.ROLE_EVAL_NU)
    counts = fi.timing_counts(ch)
    times = []
    for _ in range(reps + 1):
        t0 = time.perf_counter()
        st = m.forward(nu, ch.bias, counts)
        m.adjoint(st)
        times.append(time.perf_counter() - t0)
        del st
    med = statistics.median(times[1:])
    return {"value": 1.0 / med, "unit": "grads/s at %d^3" % n_cpu, "cores": ncpu, "kind": "oracle",
            "mesh": n_cpu, "seconds_per_gradient": med, "voxel_grads_per_s": n_cpu ** 3 / med,
            "sample": "FP64 forward+adjoint of the same model (%d webs, %d regions, RSD, same cell size) at "
                      "%d^3, L=%g: median of %d runs after one warm-up (%s s)" % (
                          ws.web.n_webs, ws.n_regions, n_cpu, ch.box, reps,
                          ", ".join("%.2f" % t for t in times[1:]))}


def copy_calibration(torch, gib=1, reps=5):
    """A plain device-to-device copy of known size: the reference that scales
    the FETCH_SIZE / WRITE_SIZE counters to bytes."""
    nbytes = gib << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": nbytes, "bytes_written": nbytes, "launches": reps}}),
          flush=True)


def _sampling_state(plan, w, torch):
    """A state a sampler would visit, for timing runs that move it: every
    chain at its truth noise, with counts drawn from the model's own mean
    there (this plan's forward model on cheap timing counts, then
    Gamma-Poisson draws with the region-0 dispersion).  There the gradient is
    O(1) per mode, so a trajectory keeps the fields and particle displacements
    of the start.  (Away from the data, e.g. at an independent noise draw,
    tracers sit in nearly empty cells, the gradient reaches 1e8-1e11, and any
    trajectory flings the state far out: particles then land far from their
    lattice cells and the deposit costs several times more.)  Returns the
    device noise."""
    import numpy as np
    import fzw_inputs as fi
    for c, ch in enumerate(w.chains):
        plan.set_counts(c, torch.from_numpy(fi.timing_counts(ch).view(np.int16)).cuda())
    nu = torch.from_numpy(np.concatenate([fi.white_noise(ch, fi.ROLE_TRUTH_NU).astype(np.float32).ravel()
                                          for ch in w.chains])).cuda()
    base = torch.from_numpy(np.stack([ch.bias for ch in w.chains]).astype(np.float32)).cuda()
    _, nbar = plan.forward(nu, base, want_nbar=True)
    nb = nbar.cpu().numpy()
    del nbar
    for c, ch in enumerate(w.chains):
        o = plan.offsets[c]
        m = nb[o:o + ch.n ** 3].astype(np.float64)
        cnt = fi.gamma_poisson_counts(m, np.full_like(m, float(ch.bias[0, fi.COL_BETA])),
                                      fi.rng_for(ch, fi.ROLE_DATA))
        plan.set_counts(c, torch.from_numpy(cnt.view(np.int16)).cuda())
    return nu


def _trajectory(w, steps, reps, torch, Plan, CosmoParams, WebParams, step_size=1e-3, checkpoint=False):
    """Time graph-captured leapfrog trajectories of every chain of workload w
    (ragged meshes allowed): returns ms per leapfrog step (one gradient of
    every chain) over `reps` trajectories after one warm-up trajectory, and
    the workspace and the largest relative change of H over the last one.
    The state is one a sampler visits (`_sampling_state`), and the step keeps
    H to ~1e-7 relative (at 1e-2 the stiffest modes of the 128^3 chains are
    unstable)."""
    import numpy as np
    import fzw_inputs as fi
    plan = _plan(w, w.chains, Plan, CosmoParams, WebParams, checkpoint)
    nu = _sampling_state(plan, w, torch)
    mu, sig = fi.prior_arrays(w)
    plan.set_sampling(fi.tie_array(w), mu, sig)
    u = torch.from_numpy(np.stack([fi.free_start(w, ch) for ch in w.chains]).astype(np.float32)).cuda()
    base = torch.from_numpy(np.stack([ch.bias for ch in w.chains]).astype(np.float32)).cuda()
    g = np.random.default_rng(7)
    p_nu = torch.from_numpy(g.standard_normal(nu.numel()).astype(np.float32)).cuda()
    p_u = torch.from_numpy(g.standard_normal(tuple(u.shape)).astype(np.float32)).cuda()
    minv = torch.ones_like(nu)
    minv_u = torch.full_like(u, 1e-2)
    step = torch.full((len(w.chains),), step_size, dtype=torch.float32, device="cuda")
    plan.leapfrog(nu, u, p_nu, p_u, base, minv, minv_u, step, steps)     # capture + first replay
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(plan.stream)
    for _ in range(reps):
        h0, h1 = plan.leapfrog(nu, u, p_nu, p_u, base, minv, minv_u, step, steps)
    ev1.record(plan.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / (reps * steps)
    dh = float(((h1 - h0).abs() / h0.abs()).max())
    ws = plan.workspace_bytes
    del plan
    torch.cuda.empty_cache()
    return ms, ws, dh


def _nuts_leg(w, md, reps, torch, Plan, CosmoParams, WebParams, step_size=1e-4):
    """Time no-U-turn transitions of every chain of workload w, at a state a
    sampler visits (`_sampling_state`) and a step so small that no trajectory
    turns or diverges, so every transition builds the full tree of 2^md - 1
    leaves: the cost per leaf, next to a plain leapfrog step, is the tree's
    bookkeeping overhead (checkpoints, U-turn dot products, candidate copies,
    per-doubling host checks)."""
    import numpy as np
    import fzw_inputs as fi
    from paper_2506_03969_amd import nuts_n_uniforms
    plan = _plan(w, w.chains, Plan, CosmoParams, WebParams)
    nu = _sampling_state(plan, w, torch)
    mu, sig = fi.prior_arrays(w)
    plan.set_sampling(fi.tie_array(w), mu, sig)
    u = torch.from_numpy(np.stack([fi.free_start(w, ch) for ch in w.chains]).astype(np.float32)).cuda()
    base = torch.from_numpy(np.stack([ch.bias for ch in w.chains]).astype(np.float32)).cuda()
    minv = torch.ones_like(nu)
    minv_u = torch.full_like(u, 1e-2)
    step = torch.full((len(w.chains),), step_size, dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    draws = []
    for _ in range(reps + 1):
        draws.append((torch.randn(nu.numel(), generator=gen, device="cuda"),
                      torch.randn(tuple(u.shape), generator=gen, device="cuda"),
                      torch.rand((len(w.chains), nuts_n_uniforms(md)), generator=gen, device="cuda")))
    plan.nuts(nu, u, *draws[0][:2], base, minv, minv_u, step, draws[0][2], md)      # allocates the state
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    leaves = []
    ev0.record(plan.stream)
    for r in range(reps):
        z, zu, uni = draws[r + 1]
        pot, acc, st = plan.nuts(nu, u, z, zu, base, minv, minv_u, step, uni, md)
        leaves.append(st[:, 1].clone())
    ev1.record(plan.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    lv = torch.stack(leaves).float()
    del plan
    torch.cuda.empty_cache()
    return {"chains": len(w.chains), "max_depth": md, "transitions": reps,
            "leaves_per_transition": float(lv.mean()), "ms_per_transition": ms,
            "ms_per_leaf": ms / float(lv.max(dim=1).values.mean()),
            "chain_grads_per_s": float(lv.sum(dim=1).mean()) * 1e3 / ms}


def _hbm_measured(n, ms_per_step):
    b = measured_gradient_traffic(n)
    if b is None:
        return None
    return {"bytes_per_gradient": b, "GBps": b / (ms_per_step * 1e6), "peak": HBM_PEAK_GBS,
            "frac": b / (ms_per_step * 1e6) / HBM_PEAK_GBS,
            "source": "profiles/traffic_gradient_%d.json (rocprofv3 FETCH_SIZE + WRITE_SIZE over every kernel, "
                      "scaled by a 1 GiB copy)" % n}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-trajectories", action="store_true",
                    help="skip the ragged 32-chain and the 512^3 leapfrog trajectories")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (for scaling HBM byte counters)")
    ap.add_argument("--gradients-only", type=int, default=0,
                    help="only create the plan and run this many forward+adjoint evaluations (byte counters)")
    ap.add_argument("--trajectory-only", default="",
                    help="only run this workload's graph-captured trajectories (c3 or c4; for kernel traces)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: it measures the single-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if args.copy_calibration:
        copy_calibration(torch)
        return
    if args.gradients_only > 0:
        gradients_only(args.gradients_only, args.workload, torch)
        return
    if args.trajectory_only:
        import fzw_inputs as fi
        from paper_2506_03969_amd import CosmoParams, Plan, WebParams
        wt = fi.workload(args.trajectory_only)
        ms, ws, dh = _trajectory(wt, wt.leapfrog_steps, 2, torch, Plan, CosmoParams, WebParams)
        print(json.dumps({"trajectory_only": args.trajectory_only, "ms_per_leapfrog_step": ms, "max_rel_dH": dh}),
              flush=True)
        return
    import fzw_inputs as fi
    from paper_2506_03969_amd import CosmoParams, Plan, WebParams, fft_schedule

    w = fi.workload(args.workload)
    ch = w.chains[0]
    n = ch.n
    print("# workload %s: %d^3, L=%g, webs=%d, regions=%d, rsd_axis=%d" % (
        w.name, n, ch.box, w.web.n_webs, w.n_regions, w.cosmo.rsd_axis), file=sys.stderr, flush=True)
    nu_h = fi.white_noise(ch, fi.ROLE_EVAL_NU).astype(np.float32)
    counts_h = fi.timing_counts(ch)
    plan = _plan(w, [ch], Plan, CosmoParams, WebParams)
    plan.set_counts(0, torch.from_numpy(counts_h.view(np.int16)).cuda())
    schedule = {k: {"family": v[0], "us_four_step": v[1], "us_alternative": v[2]}
                for k, v in fft_schedule(n).items()}
    nu = torch.from_numpy(nu_h.ravel()).cuda()
    bias = torch.from_numpy(ch.bias.astype(np.float32)[None]).cuda()
    out = (torch.empty(1, dtype=torch.float64, device="cuda"), torch.empty_like(nu), torch.empty_like(bias))
    for _ in range(args.warmup):
        plan.value_and_grad(nu, bias, out)
    torch.cuda.synchronize()
    print("# warmup done", file=sys.stderr, flush=True)
    gpu_s, wall = _time_steps(plan, nu, bias, out, args.steps, torch)
    ms_per_step = 1e3 * gpu_s / args.steps
    value = args.steps / gpu_s
    print("# single chain: %.3f ms/step (wall %.3f ms/step)" % (ms_per_step, 1e3 * wall / args.steps),
          file=sys.stderr, flush=True)

    # per-kernel-class HIP-event timing over a second timed region
    plan.timing(True)
    _time_steps(plan, nu, bias, out, args.steps, torch)
    rep = plan.timing_report()
    plan.timing(False)
    classes = {}
    for k, (ms, launches, by) in rep.items():
        if launches:
            classes[k] = {"ms_per_step": ms / args.steps, "launches_per_step": launches / args.steps,
                          "avg_launch_us": 1e3 * ms / launches, "GBps": by / (ms * 1e6) if ms > 0 else 0.0}
    # the dominant kernel: the single-kernel class with the most time
    from paper_2506_03969_amd.fzw import SINGLE_KERNEL_CLASSES
    dom = max(((k, v) for k, v in rep.items() if k in SINGLE_KERNEL_CLASSES), key=lambda kv: kv[1][0])
    dom_ms, dom_n, dom_b = dom[1]
    achieved = dom_b / (dom_ms * 1e6)
    traffic = measured_traffic(dom[0], n)
    total_alg = sum(v[2] for v in rep.values()) / args.steps
    for k, v in sorted(classes.items(), key=lambda kv: -kv[1]["ms_per_step"]):
        print("#   %-11s %7.3f ms/step %6.1f launches  %8.1f us/launch  %7.1f GB/s" % (
            k, v["ms_per_step"], v["launches_per_step"], v["avg_launch_us"], v["GBps"]), file=sys.stderr)

    # the alternative CIC deposit (fixed-point atomics), same results
    plan.set_cic_method("atomic")
    for _ in range(max(1, args.warmup)):
        plan.value_and_grad(nu, bias, out)
    ga, _ = _time_steps(plan, nu, bias, out, args.steps, torch)
    plan.set_cic_method("sorted")
    cic_atomic = {"ms_per_step": 1e3 * ga / args.steps, "value": args.steps / ga, "unit": "grads/s"}
    print("# with the atomic CIC deposit: %.3f ms/step" % cic_atomic["ms_per_step"], file=sys.stderr, flush=True)

    # batched: several identical 256^3 chains in one plan
    batched = None
    if args.batch > 1:
        del plan, out
        torch.cuda.empty_cache()
        chains = [ch] * args.batch
        pb = _plan(w, chains, Plan, CosmoParams, WebParams)
        for c in range(args.batch):
            pb.set_counts(c, torch.from_numpy(counts_h.view(np.int16)).cuda())
        nub = nu.repeat(args.batch)
        biasb = bias.repeat(args.batch, 1, 1).contiguous()
        outb = (torch.empty(args.batch, dtype=torch.float64, device="cuda"), torch.empty_like(nub),
                torch.empty_like(biasb))
        for _ in range(max(1, args.warmup)):
            pb.value_and_grad(nub, biasb, outb)
        bs = max(2, args.steps // args.batch)
        gb, _ = _time_steps(pb, nub, biasb, outb, bs, torch)
        batched = {"chains": args.batch, "value": args.batch * bs / gb, "unit": "grads/s",
                   "ms_per_step": 1e3 * gb / bs}
        print("# batched x%d: %.3f ms/step -> %.1f grads/s" % (args.batch, batched["ms_per_step"],
                                                              batched["value"]), file=sys.stderr)
        del pb
        torch.cuda.empty_cache()

    # leapfrog trajectories (hipGraph per trajectory): 32 ragged chains, and 512^3
    trajectories = None
    if not args.no_trajectories:
        trajectories = {}
        for name, ck in (("c3", False), ("c4", False), ("c4", True)):
            wt = fi.workload(name)
            ms, ws, dh = _trajectory(wt, wt.leapfrog_steps, 2, torch, Plan, CosmoParams, WebParams, checkpoint=ck)
            vox = sum(ch.n ** 3 for ch in wt.chains)
            model = sum(fi.bytes_model(ch.n, wt.web.n_webs, leapfrog=True) for ch in wt.chains)
            trajectories[name + ("_checkpointed" if ck else "")] = {
                "chains": len(wt.chains), "meshes": sorted({ch.n for ch in wt.chains}),
                "leapfrog_steps": wt.leapfrog_steps, "ms_per_leapfrog_step": ms, "workspace_bytes": ws,
                "state": "truth noise, counts drawn from the model there; step 1e-3", "max_rel_dH": dh,
                "grads_per_s": len(wt.chains) * 1e3 / ms, "voxel_grads_per_s": vox * 1e3 / ms,
                "model_GBps": model / (ms * 1e6), "hbm_frac_model": model / (ms * 1e6) / HBM_PEAK_GBS}
            print("# %s%s trajectory: %d chains, %.3f ms per leapfrog step (%.1f grads/s, %.0f GB/s model), "
                  "workspace %.1f GB" % (name, " checkpointed" if ck else "", len(wt.chains), ms,
                                         len(wt.chains) * 1e3 / ms, model / (ms * 1e6), ws / 1e9),
                  file=sys.stderr, flush=True)

    # batched vs single where batching matters: each c3 mesh size alone (one
    # chain, the same 10-step graph trajectory), and the 32 chains run one
    # after another at those rates, against the batched trajectory above
    c3_single = None
    if not args.no_trajectories and trajectories and "c3" in trajectories:
        import dataclasses
        wt = fi.workload("c3")
        per = {}
        for n_ in sorted({ch.n for ch in wt.chains}):
            ch1 = next(ch for ch in wt.chains if ch.n == n_)
            ms1, _, _ = _trajectory(dataclasses.replace(wt, chains=[ch1]), wt.leapfrog_steps, 2, torch, Plan,
                                    CosmoParams, WebParams)
            per[n_] = ms1
        seq_ms = sum(per[ch.n] for ch in wt.chains)
        c3_single = {"ms_per_leapfrog_step_alone": {str(k): v for k, v in per.items()},
                     "sequential_ms_per_step_all_chains": seq_ms,
                     "batched_ms_per_step_all_chains": trajectories["c3"]["ms_per_leapfrog_step"],
                     "batched_over_sequential_rate": seq_ms / trajectories["c3"]["ms_per_leapfrog_step"]}
        print("# c3 alone per leapfrog step: %s ms; the 32 chains in sequence %.2f ms vs batched %.2f ms (x%.2f)" % (
            ", ".join("%d^3 %.3f" % kv for kv in per.items()), seq_ms, trajectories["c3"]["ms_per_leapfrog_step"],
            c3_single["batched_over_sequential_rate"]), file=sys.stderr, flush=True)

    # no-U-turn transitions of the 32 ragged chains (full trees of 31 leaves)
    nuts_leg = None
    if not args.no_trajectories:
        wt = fi.workload("c3")
        nuts_leg = _nuts_leg(wt, 5, 3, torch, Plan, CosmoParams, WebParams)
        nuts_leg["workload"] = "c3: 32 chains (12 x 64^3, 10 x 96^3, 10 x 128^3)"
        if trajectories and "c3" in trajectories:
            nuts_leg["leaf_vs_leapfrog_step"] = nuts_leg["ms_per_leaf"] / trajectories["c3"]["ms_per_leapfrog_step"]
        print("# c3 NUTS: %.2f ms per transition of %.0f leaves, %.3f ms per leaf (%.1f chain-grads/s)" % (
            nuts_leg["ms_per_transition"], nuts_leg["leaves_per_transition"], nuts_leg["ms_per_leaf"],
            nuts_leg["chain_grads_per_s"]), file=sys.stderr, flush=True)

    # validation statistics of a 256^3 field (multipoles, 32 shells; reduced
    # bispectrum at k1 = 0.1, k2 = 0.2 h/Mpc over 9 opening angles)
    stats_leg = None
    if not args.no_trajectories:
        ps = _plan(w, [ch], Plan, CosmoParams, WebParams)
        delta = torch.from_numpy(fi.white_noise(ch, fi.ROLE_MISC).astype(np.float32).ravel()).cuda()
        kf = 2 * np.pi / ch.box
        thetas = list(np.linspace(0.05, np.pi - 0.05, 9))
        ps.power_multipoles(delta, None, k_lo=kf, dk=kf, nbins=32, mesh_n=n)
        ps.bispectrum(delta, 0.1, 0.2, 2 * kf, thetas, mesh_n=n)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(ps.stream)
        for _ in range(5):
            ps.power_multipoles(delta, None, k_lo=kf, dk=kf, nbins=32, mesh_n=n)
        e1.record(ps.stream)
        torch.cuda.synchronize()
        ms_pk = e0.elapsed_time(e1) / 5
        e0.record(ps.stream)
        ps.bispectrum(delta, 0.1, 0.2, 2 * kf, thetas, mesh_n=n)
        e1.record(ps.stream)
        torch.cuda.synchronize()
        stats_leg = {"mesh": n, "multipoles_ms": ms_pk, "multipole_shells": 32,
                     "bispectrum_ms": e0.elapsed_time(e1), "bispectrum_angles": len(thetas)}
        print("# statistics at %d^3: P0/P2 %.3f ms, bispectrum (9 angles) %.3f ms" % (
            n, ms_pk, stats_leg["bispectrum_ms"]), file=sys.stderr, flush=True)
        del ps
        torch.cuda.empty_cache()

    cpu = None if args.no_cpu else cpu_baseline(w)
    model_bytes = fi.bytes_model(n, w.web.n_webs)
    line = {
        "metric": "forward+adjoint logL grads/sec at 256^3 (FP32, batched vs single) + % HBM peak",
        "value": value,
        "unit": "grads/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s: %d^3 mesh, L=%g Mpc/h, %d webs, %d regions, plane-parallel RSD, "
                               "1 chain, forward+adjoint" % (w.name, n, ch.box, w.web.n_webs, w.n_regions),
                   "mesh": n, "box": ch.box, "chains": 1},
        "batched": batched,
        "cic_atomic": cic_atomic,
        "hbm_measured": _hbm_measured(n, ms_per_step),
        "model_bytes_per_grad": model_bytes,
        "model_GBps": model_bytes / (ms_per_step * 1e6),
        "hbm_frac_model": model_bytes / (ms_per_step * 1e6) / HBM_PEAK_GBS,
        "trajectories": trajectories,
        "c3_batched_vs_single": c3_single,
        "nuts": nuts_leg,
        "statistics": stats_leg,
        "algorithmic_GBps_all_kernels": total_alg / (ms_per_step * 1e6),
        "hbm_frac_algorithmic": total_alg / (ms_per_step * 1e6) / HBM_PEAK_GBS,
        "kernel_classes": classes,
        "fft_schedule": schedule,
        "roofline": {"bound": "hbm", "kernel": dom[0], "symbol": KERNEL_SYMBOLS.get(dom[0], "").format(n=n, w=w.web.n_webs),
                     "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": dom_b / dom_n,
                     "avg_launch_us": 1e3 * dom_ms / dom_n},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
