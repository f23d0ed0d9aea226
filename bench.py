#!/usr/bin/env python
"""Benchmark of the pressure-projection solve on one MI355X.

Workload: the 256^3 rising-bubble sequence (radius 0.1 starting at (0.5, 0.5, 0.2),
+0.004 in z per step, density ratio 1000, sigma = 0.01, Neumann walls, one seeded
uniform right-hand side per step).  One step = one projection solve: build the
operator for that step's level set and solve to a relative residual of 1e-10,
warm-started from the previous step's pressure.  Inputs (phi_t, f_t) for every
step are resident in HBM before the timed region.

Methods run on the same steps:
  plain   -- FP64 multigrid-preconditioned CG warm-started from the previous step's
             pressure (the baseline: no deflation),
  plain0  -- the same from a zero initial guess,
  plain_d -- plain with the bubble regions deflated,
  mixed   -- FP32 multigrid-preconditioned CG inside FP64 residual refinement, deflated,
             warm started likewise,
  mixed0  -- mixed from a zero initial guess,
  learned -- mixed, started from the learned guess: the U-Net trained on 64^3 problems
             (weights shipped with the package) applied to the step's inputs averaged
             over 4^3 blocks, its prediction prolonged to 256^3, scaled to the energy
             optimum and smoothed by two red-black sweeps.
The headline value is the learned method's mean time per step (ms, lower is better);
the others are reported beside it with the speed-up over plain.

Also reported: the dominant kernel's achieved HBM bandwidth (algorithmic bytes per
launch / mean launch time from HIP events in a profiled repeat of the timed steps),
and the CPU oracle timed on the host cores on a bounded sample (one full-size solve).

Other workloads (--workload) measure the steps around the solve, the heat step, the
block layout and the two-level composite grid, each with the oracle timed beside it.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib

import numpy as np
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
NU_COARSE = 0   # sweeps per level below the finest (0: as the finest); set by --nu-coarse


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_sha():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2312_11740_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were taken
    on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    rec = t.get(kernel)
    if not rec or rec.get("src_sha") != kernel_sources_sha():
        return None
    return rec.get("bytes_per_launch")


def run_sequence(M, torch, ws, phis, fs, prm, mode, nu, steps, warmup, net=None, zero=False,
                 guess_sweeps=2, check_every=2, deflate=True):
    """warmup + steps projection solves, each warm-started from the previous step (or,
    with a network, from the learned guess; with zero, from zero); returns (mean ms per
    timed step, infos of the timed steps, learned-guess fallbacks)."""
    p = torch.zeros_like(fs[0])
    infos = []
    fallbacks = 0
    t0 = None
    op = M.Operator(phis[0], prm["rho_neg"], prm["rho_pos"], prm["sigma"], workspace=ws)
    for t in range(warmup + steps):
        if t == warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        op.update(phis[t], prm["rho_neg"], prm["rho_pos"], prm["sigma"])
        start_zero = zero
        if net is not None:
            p, fell = op.learned_guess(net, fs[t], sweeps=guess_sweeps, out=p,
                                       judge="deflated" if deflate else "plain")
            if t >= warmup:
                fallbacks += sum(fell)
            # a guess replaced by zero: the solve starts from zero (p is only its output)
            start_zero = all(fell)
        p, info = op.solve(fs[t], p=p, zero=start_zero, rtol=prm["rtol"], mode=mode, nu=nu,
                           nu_coarse=NU_COARSE, check_every=check_every, deflate=deflate,
                           reuse_rhs=net is not None)
        if t >= warmup:
            infos.append(info[0])
    torch.cuda.synchronize()
    op.close()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return ms, infos, fallbacks


def run_profiled(M, torch, ws, phis, fs, prm, mode, nu, steps, warmup, net=None, zero=False,
                 deflate=True):
    p = torch.zeros_like(fs[0])
    stats = {}
    op = M.Operator(phis[0], prm["rho_neg"], prm["rho_pos"], prm["sigma"], workspace=ws)
    for t in range(warmup + steps):
        op.update(phis[t], prm["rho_neg"], prm["rho_pos"], prm["sigma"])
        start_zero = zero
        if net is not None:
            p, fell = op.learned_guess(net, fs[t], sweeps=2, out=p,
                                       judge="deflated" if deflate else "plain")
            start_zero = all(fell)
        if t >= warmup:
            op.profile_start()
        p, info = op.solve(fs[t], p=p, zero=start_zero, rtol=prm["rtol"], mode=mode, nu=nu,
                           nu_coarse=NU_COARSE, deflate=deflate, reuse_rhs=net is not None)
        if t >= warmup:
            for k, v in op.profile_stop().items():
                s = stats.setdefault(k, dict(launches=0, ms=0.0, bytes=0.0))
                for f in ("launches", "ms", "bytes"):
                    s[f] += v[f]
    torch.cuda.synchronize()
    op.close()
    return stats


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(prob, p_gpu):
    """The FP64 CPU oracle (as it stands) on one full-size step: assemble + MG-PCG to
    1e-10 on the host cores.  Returns the record and the GPU-vs-oracle error."""
    import numpy as np
    import oracle as O
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    d = O.pipeline(prob.phi, prob.f, prob.rho_neg, prob.rho_pos, prob.sigma)
    po, oi = O.solve_mg_pcg(d["faces"], d["b"], tol=1e-10)
    sec = time.perf_counter() - t0
    err = None
    rr = None
    if p_gpu is not None:
        err = float(np.linalg.norm(p_gpu - po) / np.linalg.norm(po))
        rr = float(O.rel_residual(d["faces"], d["b"], p_gpu))
    rec = {"value": round(sec * 1e3, 1), "unit": "ms", "cores": cores, "cpu": cpu_model(),
           "kind": "oracle",
           "sample": "one 256^3 step (t=0) of the same sequence, zero start, assemble + "
                     "FP64 MG-PCG (nu=2) to 1e-10 (%d iterations)" % oi["iters"]}
    return rec, err, rr


def copy_calibration(torch, nbytes):
    """A plain device copy of known size, for scaling HBM counters."""
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 10
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8,
                      "ms": dt * 1e3, "GBps": 2 * n * 8 / dt / 1e9}), flush=True)


def batched64(M, G, torch, args):
    """64 independent 64^3 bubble problems (count 1..8, ratio 10..1000, seeds 20000..20063)
    solved together: time per batch (operator build + solve to 1e-10, zero start)."""
    dev = torch.device("cuda:0")
    n, B = 64, 64
    log("generating %d problems of %d^3" % (B, n))
    probs = [G.random_bubbles_problem(20000 + s, n=n) for s in range(B)]
    phi = torch.from_numpy(np.stack([q.phi for q in probs])).to(dev)
    f = torch.from_numpy(np.stack([q.f for q in probs])).to(dev)
    rn = [q.rho_neg for q in probs]
    rp = [q.rho_pos for q in probs]
    sg = [q.sigma for q in probs]
    op = M.Operator(phi, rn, rp, sg)
    res = {}
    for meth, mode, dfl, tail in (("plain", "fp64", False, True),
                                  ("plain_d", "fp64", True, True),
                                  ("plain_d_notail", "fp64", True, False),
                                  ("mixed_nd", "mixed", False, True),
                                  ("mixed", "mixed", True, True),
                                  ("mixed_notail", "mixed", True, False)):
        # the tail schedule (sweep tiles tuned for one live problem) takes over once at
        # most 8 of the 64 problems are still iterating; *_notail keeps the batch schedule
        os.environ["MPP_TAIL"] = "1" if tail else "0"
        for _ in range(args.warmup):
            op.update(phi, rn, rp, sg)
            op.solve(f, rtol=1e-10, mode=mode, nu=args.nu, deflate=dfl)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            op.update(phi, rn, rp, sg)
            p, infos = op.solve(f, rtol=1e-10, mode=mode, nu=args.nu, deflate=dfl)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        its = [i.iters for i in infos]
        res[meth] = {"ms_per_batch": round(ms, 3),
                     "iters_max": max(its),
                     "iters_mean": sum(its) / B,
                     # problems still iterating at each (inner, for mixed) CG iteration
                     "active_per_iter": [sum(k < i for i in its) for k in range(max(its))],
                     "max_rel_resid": max(i.rel_resid for i in infos),
                     "ok": all(i.status == M.OK for i in infos)}
        log(meth, res[meth])
    os.environ.pop("MPP_TAIL", None)
    best = min(res, key=lambda m: res[m]["ms_per_batch"])
    print(json.dumps({"metric": "time per batch of 64 x 64^3 solves to 1e-10", "value":
                      res[best]["ms_per_batch"], "unit": "ms", "higher_is_better": False,
                      "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "data": "synthetic", "config": {"workload": "batched 64 x 64^3 bubbles",
                                                      "method": best},
                      "methods": res}), flush=True)


def cpu_baseline_single(pr, solutions, rtol):
    """The CPU leg of a single-problem workload: the oracle (assemble + its FP64 MG-PCG to
    1e-13) timed on the host cores, and each GPU method's error against its solution."""
    import oracle as O
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    po, _, oi = O.solve(pr.phi, pr.f, pr.rho_neg, pr.rho_pos, pr.sigma, tol=1e-13)
    sec = time.perf_counter() - t0
    errs = {m: float(np.linalg.norm(ph - po) / np.linalg.norm(po)) for m, ph in solutions.items()}
    rec = {"value": round(sec * 1e3, 1), "unit": "ms", "cores": cores, "cpu": cpu_model(),
           "kind": "oracle",
           "sample": "the whole problem: assemble + FP64 MG-PCG (nu=2) to 1e-13 (%d iterations)"
                     % oi["iters"]}
    return rec, errs


def single_problem(M, G, torch, args, which):
    """One of the fixed single-problem configurations, plain vs mixed, zero start:
    single32 -- one sphere r 0.25 at the centre, rho 1 inside / 10 outside, sigma 0,
                manufactured right-hand side, 32^3;
    bubbles128 -- 20 bubbles (seed 1, r in [0.04, 0.12]), ratio 1000, sigma 0.01, 128^3.
    Time per solve (operator built once, outside the timed region), iterations and the
    error against the oracle's solution."""
    dev = torch.device("cuda:0")
    pr = G.single_bubble_problem(32) if which == "single32" else G.many_bubbles_problem()
    rtol = 1e-10 if which == "single32" else 2e-11
    phi = torch.from_numpy(pr.phi).to(dev)
    f = torch.from_numpy(pr.f).to(dev)
    op = M.Operator(phi, pr.rho_neg, pr.rho_pos, pr.sigma)
    res, sols = {}, {}
    for meth, mode, dfl in (("plain", "fp64", False), ("plain_d", "fp64", True),
                            ("mixed_nd", "mixed", False), ("mixed", "mixed", True)):
        for _ in range(args.warmup):
            op.solve(f, rtol=rtol, mode=mode, nu=args.nu, deflate=dfl)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            p, infos = op.solve(f, rtol=rtol, mode=mode, nu=args.nu, deflate=dfl)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        sols[meth] = p.cpu().numpy()
        res[meth] = {"ms_per_solve": round(ms, 3), "iters": infos[0].iters,
                     "outer": infos[0].outer_iters, "rel_resid": infos[0].rel_resid,
                     "ok": infos[0].status == M.OK}
        log(meth, res[meth])
    cpu = None
    if not args.no_cpu_baseline:
        cpu, errs = cpu_baseline_single(pr, sols, rtol)
        for m in res:
            res[m]["err_vs_oracle"] = errs[m]
        log("cpu baseline", cpu, errs)
    best = min(res, key=lambda m: res[m]["ms_per_solve"])
    print(json.dumps({"metric": "time per solve to %g rel. residual" % rtol,
                      "value": res[best]["ms_per_solve"], "unit": "ms",
                      "higher_is_better": False, "n_gpus": 1, "steps": args.steps,
                      "warmup": args.warmup, "data": "synthetic",
                      "config": {"workload": which, "method": best},
                      "methods": res, "cpu_baseline": cpu}), flush=True)


def oracle_leg(fn, sample):
    """Times one run of an oracle computation on the host cores; returns (the
    cpu_baseline record, the computation's result)."""
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    out = fn()
    sec = time.perf_counter() - t0
    rec = {"value": round(sec * 1e3, 1), "unit": "ms", "cores": cores, "cpu": cpu_model(),
           "kind": "oracle", "sample": sample}
    return rec, out


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def projection256(M, G, torch, args):
    """The projection step around the solve on the 256^3 rising-bubble sequence: f =
    div(u*)/dt from seeded face velocities, the mixed solve warm-started from the
    previous step, the jump-consistent correction.  Time per step and the HIP-event time
    of the divergence and correction kernels against the HBM roofline."""
    dev = torch.device("cuda:0")
    n, K, W = 256, args.steps, args.warmup
    prm = dict(rho_neg=1e-3, rho_pos=1.0, sigma=0.01)
    dt = 1e-3
    probs = [G.rising_bubble_problem(t, n=n) for t in range(K + W)]
    phis = [torch.from_numpy(q.phi).to(dev) for q in probs]
    gen = torch.Generator(device=dev)
    gen.manual_seed(50000)
    us = []
    for _ in range(K + W):
        u = [torch.randn((n, n, n), dtype=torch.float64, device=dev, generator=gen)
             for _ in range(3)]
        u[0][:, :, 0] = 0.0
        u[1][:, 0, :] = 0.0
        u[2][0, :, :] = 0.0
        us.append(u)
    u0_host = [a.cpu().numpy() for a in us[0]]   # step 0's predicted velocity, for the oracle
    op = M.Operator(phis[0], **prm)
    p = torch.zeros((n, n, n), dtype=torch.float64, device=dev)
    f = torch.empty_like(p)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    t_div, t_proj = [], []
    for t in range(K + W):
        if t == W:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        op.update(phis[t], **prm)
        ev[0].record()
        op.divergence(us[t], dt, out=f)
        ev[1].record()
        # mixed solve warm-started from the previous step's pressure, without deflation:
        # div(u*)/dt carries no jump term for deflation to remove, and the pressure moves
        # little between steps (measured faster than a deflated solve from zero or warm)
        p, info = op.solve(f, p=p, rtol=1e-10, mode="mixed", nu=args.nu, deflate=False)
        ev[2].record()
        op.project(phis[t], p, dt, us[t])
        ev[3].record()
        if t >= W:
            torch.cuda.synchronize()
            t_div.append(ev[0].elapsed_time(ev[1]))
            t_proj.append(ev[2].elapsed_time(ev[3]))
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / K
    # divergence left after the last step relative to div(u*)/dt (still in f)
    ratio = float(torch.linalg.vector_norm(op.divergence(us[-1], dt)) /
                  torch.linalg.vector_norm(f))
    cells = n ** 3
    div_ms, proj_ms = float(np.mean(t_div)), float(np.mean(t_proj))
    div_bytes, proj_bytes = 32.0 * cells, 64.0 * cells
    rec = {"metric": "time per projection step (divergence + mixed solve + correction), 256^3",
           "value": round(ms, 3), "unit": "ms", "higher_is_better": False, "n_gpus": 1,
           "steps": K, "warmup": W, "data": "synthetic",
           "config": {"workload": "projection256", "dt": dt},
           "kernels": {"divergence": {"ms": round(div_ms, 4),
                                      "GBps": round(div_bytes / (div_ms * 1e-3) / 1e9, 1),
                                      "alg_bytes": div_bytes},
                       "project": {"ms": round(proj_ms, 4),
                                   "GBps": round(proj_bytes / (proj_ms * 1e-3) / 1e9, 1),
                                   "alg_bytes": proj_bytes}},
           "iters_last": info[0].iters, "div_ratio_last": ratio}
    if not args.no_cpu_baseline:
        import oracle as O
        q0 = probs[0]

        def step():
            fo = O.divergence(u0_host, dt)
            od = O.pipeline(q0.phi, fo, prm["rho_neg"], prm["rho_pos"], prm["sigma"])
            po, _ = O.solve_mg_pcg(od["faces"], od["b"], tol=1e-10)
            return O.project(q0.phi, od["kappa"], po, prm["rho_neg"], prm["rho_pos"], prm["sigma"],
                             dt, u0_host)
        rec["cpu_baseline"], uo = oracle_leg(step, "step 0 at full size: divergence, operator, "
                                             "FP64 MG-PCG to 1e-10 from zero, correction")
        rec["err_vs_oracle_step0"] = max(rel_err(a.cpu().numpy(), b) for a, b in zip(us[0], uo))
    print(json.dumps(rec), flush=True)


def flow256(M, G, torch, args):
    """Whole time steps of a buoyant bubble at 256^3 (density ratio 1000, sigma 0.01):
    gravity on the vertical faces, operator rebuilt from the moving level set, projection
    around the mixed solve (warm start), upwind advection of the level set by the new
    velocity and two re-distancing steps.  Time per step and the HIP-event time of the
    level-set kernels against the HBM roofline."""
    dev = torch.device("cuda:0")
    n, K, W = 256, args.steps, args.warmup
    prm = dict(rho_neg=1e-3, rho_pos=1.0, sigma=0.01)
    dt, g = 1e-3, 1.0
    phi = torch.from_numpy(G.bubble_phi(n, [(0.5, 0.5, 0.3)], [0.1])).to(dev)
    u = [torch.zeros_like(phi) for _ in range(3)]
    p = torch.zeros_like(phi)
    op = M.Operator(phi, **prm)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t_adv, t_re, iters = [], [], []
    phi0, work = torch.empty_like(phi), torch.empty_like(phi)
    zs = torch.from_numpy(((np.arange(n) + 0.5) / n)).to(dev)[:, None, None]

    def centre(ph):
        m = (ph < 0).double()
        return float((zs * m).sum() / m.sum())

    phi_init = phi.cpu().numpy()
    phi_step1 = None
    for t in range(K + W):
        if t == W:
            torch.cuda.synchronize()
            z0 = centre(phi)
            t0 = time.perf_counter()
        u[2][1:, :, :] -= dt * g
        op.update(phi, **prm)
        f = op.divergence(u, dt)
        # mixed solve warm-started from the previous step's pressure, without deflation:
        # div(u*)/dt carries no jump term for deflation to remove, and the pressure moves
        # little between steps (measured faster than a deflated solve from zero or warm)
        p, info = op.solve(f, p=p, rtol=1e-10, mode="mixed", nu=args.nu, deflate=False)
        op.project(phi, p, dt, u)
        ev[0].record()
        new = M.ls_advect(phi, u, dt)
        ev[1].record()
        phi0.copy_(new)
        M.ls_reinit(new, 2, phi0=phi0, work=work)
        ev[2].record()
        phi = new
        if t == 0 and W >= 1:
            phi_step1 = phi.cpu().numpy()   # state after step 0 (a warm-up step), for the oracle
        if t >= W:
            torch.cuda.synchronize()
            t_adv.append(ev[0].elapsed_time(ev[1]))
            t_re.append(ev[1].elapsed_time(ev[2]))
            iters.append(info[0].iters)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / K
    cells = n ** 3
    adv_ms, re_ms = float(np.mean(t_adv)), float(np.mean(t_re))
    adv_bytes, re_bytes = 40.0 * cells, 2 * 24.0 * cells
    rec = {"metric": "time per buoyant-bubble step (gravity, projection with the mixed solve, "
                     "level-set advection and re-distancing), 256^3",
           "value": round(ms, 3), "unit": "ms", "higher_is_better": False, "n_gpus": 1,
           "steps": K, "warmup": W, "data": "synthetic",
           "config": {"workload": "flow256", "dt": dt, "g": g},
           "kernels": {"ls_advect": {"ms": round(adv_ms, 4),
                                     "GBps": round(adv_bytes / (adv_ms * 1e-3) / 1e9, 1),
                                     "alg_bytes": adv_bytes},
                       "ls_reinit_x2": {"ms": round(re_ms, 4),
                                        "GBps": round(re_bytes / (re_ms * 1e-3) / 1e9, 1),
                                        "alg_bytes": re_bytes}},
           "solve_iters": iters, "bubble_rise": centre(phi) - z0}
    if not args.no_cpu_baseline and phi_step1 is not None:
        import oracle as O

        def step():
            uo = [np.zeros((n, n, n)) for _ in range(3)]
            uo[2][1:, :, :] -= dt * g
            fo = O.divergence(uo, dt)
            od = O.pipeline(phi_init, fo, prm["rho_neg"], prm["rho_pos"], prm["sigma"])
            po, _ = O.solve_mg_pcg(od["faces"], od["b"], tol=1e-10)
            uo = O.project(phi_init, od["kappa"], po, prm["rho_neg"], prm["rho_pos"], prm["sigma"],
                           dt, uo)
            new = O.ls_advect(phi_init, uo, dt)
            return O.ls_reinit(new, new, 2, 0.5 / n)
        rec["cpu_baseline"], po1 = oracle_leg(step, "step 0 at full size: gravity, divergence, "
                                              "operator, FP64 MG-PCG to 1e-10, correction, "
                                              "advection, two re-distancing steps")
        rec["err_vs_oracle_step0"] = rel_err(phi_step1, po1)
    print(json.dumps(rec), flush=True)


def heat256(M, G, torch, args):
    """Implicit diffusion steps at 256^3 on the rising-bubble interface: conductivity
    1e-2 in the liquid (phi <= 0) and 4e-4 in the vapour (ratio 25), dt 1e-2, so
    dt K_liquid / h^2 = 6.6 (a step an explicit scheme could not take); each step
    solves (I - dt div(K grad)) T = T_old in place from the previous T, to 1e-10.  The
    value is the multigrid-preconditioned mixed-precision solve; the FP64 multigrid and
    the Jacobi-preconditioned CG are timed beside it.  Kernel times come from the
    library's HIP-event profiler on one more step."""
    dev = torch.device("cuda:0")
    n, K, W = 256, args.steps, args.warmup
    kn, kp, dt = 1e-2, 4e-4, 1e-2
    phi = torch.from_numpy(G.rising_bubble_problem(0, n=n).phi).to(dev)
    op = M.Operator(phi, rho_neg=1.0 / kn, rho_pos=1.0 / kp, sigma=0.0)
    rng = np.random.default_rng(7)
    T0 = torch.from_numpy(rng.uniform(0.0, 1.0, (n, n, n))).to(dev)
    methods = {"mg_mixed": dict(precond="mg", mode="mixed"),
               "mg_fp64": dict(precond="mg", mode="fp64"),
               "jacobi": dict(precond="jacobi")}
    res = {}
    first = {}
    for name, how in methods.items():
        T = T0.clone()
        iters = []
        for t in range(K + W):
            if t == W:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            T, info = op.heat_solve(T, dt, t=T, rtol=1e-10, **how)
            if t == 0 and W >= 1:
                first[name] = T.cpu().numpy()   # step 0 (a warm-up step), for the oracle
            if t >= W:
                iters.append(info[0].iters)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / K
        op.profile_start()
        op.heat_solve(T.clone(), dt, t=T.clone(), rtol=1e-10, **how)
        stats = op.profile_stop()
        kern = {}
        for kname, st in stats.items():
            launches, total_ms, nbytes = st["launches"], st["ms"], st["bytes"]
            if launches and nbytes > 0:
                avg = total_ms / launches
                kern[kname] = {"launches": launches, "avg_us": round(avg * 1e3, 2),
                               "GBps": round(nbytes / launches / (avg * 1e-3) / 1e9, 1)}
        res[name] = {"ms_per_step": round(ms, 3), "iters": iters, "kernels": kern}
    rec = {"metric": "time per implicit heat-diffusion step (multigrid-preconditioned CG, "
                     "mixed precision, to 1e-10), 256^3",
           "value": res["mg_mixed"]["ms_per_step"], "unit": "ms",
           "higher_is_better": False, "n_gpus": 1, "steps": K, "warmup": W,
           "data": "synthetic", "dtype": "f64+f32",
           "config": {"workload": "heat256", "dt": dt, "k_liquid": kn, "k_vapour": kp},
           "methods": res}
    if not args.no_cpu_baseline:
        import oracle as O
        t0h = T0.cpu().numpy()

        def step():
            return O.heat_step(O.heat_faces(phi.cpu().numpy(), kn, kp), t0h, dt, tol=1e-10)[0]
        rec["cpu_baseline"], to = oracle_leg(step, "step 0 at full size: conductivity faces, "
                                             "conjugate gradients to 1e-10 (no preconditioner)")
        if first:
            rec["err_vs_oracle_step0"] = {k: rel_err(v, to) for k, v in first.items()}
    print(json.dumps(rec), flush=True)


def blocks256(M, G, torch, args):
    """The 256^3 rising-bubble grid in the block-structured layout: 4096 blocks of 16^3
    cells with one guard layer.  Times (HIP events over `steps` repetitions) of the
    scatter into blocks, the guard-cell fill, the block-by-block stencil and the gather,
    against the HBM roofline with their algorithmic bytes."""
    dev = torch.device("cuda:0")
    n, nb, g = 256, 16, 1
    K, W = max(args.steps, 5), args.warmup
    pr = G.rising_bubble_problem(0, n=n)
    op = M.Operator(torch.from_numpy(pr.phi).to(dev), pr.rho_neg, pr.rho_pos, pr.sigma)
    x = torch.from_numpy(np.random.default_rng(3).standard_normal((n, n, n))).to(dev)
    xb = M.blocks_scatter(x, nb, g)
    yb = torch.empty_like(xb)
    xg = torch.empty_like(x)
    P = nb + 2 * g
    nblk = (n // nb) ** 3
    cells, padded, guards = n ** 3, nblk * P ** 3, nblk * (P ** 3 - nb ** 3)
    steps = {"scatter": (lambda: M.blocks_scatter(x, nb, g, out=xb), 16.0 * cells),
             "fill_guards": (lambda: M.blocks_fill_guards(xb, n, nb, g), 16.0 * guards),
             "apply": (lambda: op.blocks_apply(xb, nb, g, out=yb), 16.0 * padded + 24.0 * cells),
             "gather": (lambda: M.blocks_gather(xb, n, nb, g, out=xg), 16.0 * cells)}
    res = {}
    for name, (fn, nbytes) in steps.items():
        for _ in range(W + 1):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(K):
            fn()
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / K
        res[name] = {"us": round(us, 2), "GBps": round(nbytes / (us * 1e-6) / 1e9, 1),
                     "alg_bytes": nbytes}
    ms = (res["fill_guards"]["us"] + res["apply"]["us"]) / 1e3
    rec = {"metric": "guard-cell fill + block stencil on the 256^3 grid in 16^3 blocks",
           "value": round(ms, 4), "unit": "ms", "higher_is_better": False, "n_gpus": 1,
           "steps": K, "warmup": W, "data": "synthetic", "dtype": "f64",
           "config": {"workload": "blocks256", "nb": nb, "guard": g, "blocks": nblk},
           "kernels": res}
    if not args.no_cpu_baseline:
        import oracle as O
        xh = x.cpu().numpy()
        fc = O.faces(pr.phi, pr.rho_neg, pr.rho_pos)

        def step():
            blk = O.blocks_fill_guards(O.blocks_scatter(xh, nb, g), n, nb, g)
            return O.blocks_apply(fc, blk, nb, g)
        rec["cpu_baseline"], yo = oracle_leg(step, "one scatter + guard fill + block stencil at "
                                             "full size (4096 blocks)")
        M.blocks_fill_guards(xb, n, nb, g)
        rec["bit_exact_vs_oracle"] = bool(np.array_equal(op.blocks_apply(xb, nb, g).cpu().numpy(), yo))
    print(json.dumps(rec), flush=True)


def amr_fill_bytes(flags, nb, g, list1):
    """Algorithmic bytes of one guard fill of the composite grid: every guard cell of
    every stored block written once (8 B) and its source read once: one value (8 B), or
    the 8 level-1 values a level-0 guard over a refined block averages (64 B)."""
    m = flags.shape[0]
    n0 = m * nb
    P = nb + 2 * g
    li = np.arange(-g, nb + g)
    L = np.stack(np.meshgrid(li, li, li, indexing="ij"), -1).reshape(-1, 3)   # k, j, i
    guard = ~np.all((L >= 0) & (L < nb), axis=1)
    L = L[guard]
    mir = lambda a, n: np.where(a < 0, -1 - a, np.where(a >= n, 2 * n - 1 - a, a))
    reads0 = 0
    for bk in range(m):
        for bj in range(m):
            for bi in range(m):
                K = mir(bk * nb + L[:, 0], n0) // nb
                J = mir(bj * nb + L[:, 1], n0) // nb
                I = mir(bi * nb + L[:, 2], n0) // nb
                reads0 += int(np.sum(np.where(flags[K, J, I] != 0, 64, 8)))
    per_block = len(L)
    return reads0 + 8 * per_block * m ** 3 + 16 * per_block * len(list1)


def amr256(M, G, torch, args):
    """The composite grid: 20 bubbles on 128^3 coarse cells in 16^3 blocks, the blocks
    within two coarse cells of an interface refined to the 256^3 spacing.  Times (HIP
    events over `steps` repetitions) of the guard fill between levels and of the
    composite operator, against the HBM roofline with their algorithmic bytes."""
    dev = torch.device("cuda:0")
    n0, nb, g = 128, 16, 1
    K, W = max(args.steps, 5), args.warmup
    pr = G.many_bubbles_problem(n=n0)
    p0, p1 = pr.phi, G.bubble_phi(2 * n0, pr.centres, pr.radii)
    flags = G.refine_near_interface(p0, nb, 2.0 / n0)
    grid = M.AmrGrid(n0, nb, g, flags, dev)
    rng = np.random.default_rng(4)
    x0, x1 = rng.standard_normal(p0.shape), rng.standard_normal(p1.shape)
    idx = torch.from_numpy(grid.list1.astype(np.int64)).to(dev)

    def blocks(v0, v1):
        b1 = M.blocks_scatter(torch.from_numpy(v1).to(dev), nb, g).index_select(0, idx)
        return M.blocks_scatter(torch.from_numpy(v0).to(dev), nb, g), b1.contiguous()
    pb = grid.fill_guards(*blocks(p0, p1))
    xb = grid.fill_guards(*blocks(x0, x1))
    yb = grid.empty()
    P = nb + 2 * g
    nref = int(flags.sum())
    leaf_blocks = grid.nblk0 - nref + grid.nblk1
    leaf_cells = leaf_blocks * nb ** 3
    steps = {"fill_guards": (lambda: grid.fill_guards(*xb),
                             amr_fill_bytes(flags, nb, g, grid.list1)),
             "apply": (lambda: grid.apply(pb, xb, pr.rho_neg, pr.rho_pos, y=yb),
                       24.0 * P ** 3 * leaf_blocks + 8.0 * P ** 3 * nref)}
    res = {}
    for name, (fn, nbytes) in steps.items():
        for _ in range(W + 1):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(K):
            fn()
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / K
        res[name] = {"us": round(us, 2), "GBps": round(nbytes / (us * 1e-6) / 1e9, 1),
                     "alg_bytes": nbytes}
    # the composite Poisson solve (b uniform in [-1, 1] on the leaves), warm-up then timed
    f0, f1 = rng.uniform(-1, 1, p0.shape), rng.uniform(-1, 1, p1.shape)
    fb = blocks(f0, f1)
    # preconditioned by the inverse diagonal, and by the two-level multigrid cycle with the
    # level-0 operator whose faces next to refined blocks come from the fine level (the one
    # reported last, whose x the oracle checks)
    coarse = grid.coarse_operator(torch.from_numpy(p0).to(dev), pb, pr.rho_neg, pr.rho_pos)
    for name, cop in (("solve_jacobi", None), ("solve", coarse)):
        for rep in range(2):
            xs = grid.empty()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xs, info = grid.solve(pb, fb, pr.rho_neg, pr.rho_pos, x=xs, rtol=1e-10, coarse=cop)
            torch.cuda.synchronize()
            solve = {"ms": round((time.perf_counter() - t0) * 1e3, 2), "iters": info.iters,
                     "rel_resid": info.rel_resid, "status": info.status,
                     "preconditioner": "two-level multigrid" if cop else "inverse diagonal"}
        solve["ms_per_iter"] = round(solve["ms"] / max(solve["iters"], 1), 4)
        res[name] = solve
    ms = (res["fill_guards"]["us"] + res["apply"]["us"]) / 1e3
    ap = res["apply"]
    rec = {"metric": "guard fill + composite operator on a two-level grid (128^3 coarse, "
                     "256^3 spacing around the interfaces)",
           "value": round(ms, 4), "unit": "ms", "higher_is_better": False, "n_gpus": 1,
           "steps": K, "warmup": W, "data": "synthetic", "dtype": "f64",
           "config": {"workload": "amr256", "n0": n0, "nb": nb, "guard": g, "bubbles": 20,
                      "refined_level0_blocks": nref, "level1_blocks": grid.nblk1,
                      "leaf_cells": leaf_cells},
           "kernels": res,
           "roofline": {"bound": "hbm", "kernel": "k_amr_apply", "achieved": ap["GBps"],
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(ap["GBps"] / HBM_PEAK_GBS, 3), "traffic": None}}
    if not args.no_cpu_baseline:
        import oracle as O

        def step():
            O.amr_fill(flags, nb, g, x0, x1)
            return O.amr_apply(flags, nb, p0, p1, x0, x1, pr.rho_neg, pr.rho_pos)
        rec["cpu_baseline"], (e0_, e1_) = oracle_leg(step, "one guard fill + composite "
                                                     "operator at full size")
        grid.apply(pb, xb, pr.rho_neg, pr.rho_pos, y=yb)
        sel = grid.list1.astype(np.int64)
        ok0 = np.array_equal(yb[0].cpu().numpy(), O.blocks_scatter(e0_, nb, g))
        ok1 = np.array_equal(yb[1].cpu().numpy(), O.blocks_scatter(e1_, nb, g)[sel])
        rec["bit_exact_vs_oracle"] = bool(ok0 and ok1)
        # the solve's residual recomputed by the oracle from the GPU solution, and the
        # oracle's own solver timed over a bounded number of iterations
        full1 = np.zeros(((2 * n0 // nb) ** 3, P, P, P))
        full1[sel] = xs[1].cpu().numpy()
        gx0 = O.blocks_gather(xs[0].cpu().numpy(), n0, nb, g)
        gx1 = O.blocks_gather(full1, 2 * n0, nb, g)
        m0 = ~np.repeat(np.repeat(np.repeat(flags, nb, 0), nb, 1), nb, 2).astype(bool)
        m1 = np.repeat(np.repeat(np.repeat(flags, 2 * nb, 0), 2 * nb, 1), 2 * nb, 2).astype(bool)
        gx0, gx1 = np.where(m0, gx0, 0.0), np.where(m1, gx1, 0.0)
        v0, v1 = 1.0 / n0 ** 3, 1.0 / (2 * n0) ** 3
        mean = v0 * f0[m0].sum() + v1 * f1[m1].sum()
        a0, a1 = O.amr_apply(flags, nb, p0, p1, gx0, gx1, pr.rho_neg, pr.rho_pos)
        r0, r1 = np.where(m0, f0 - mean - a0, 0.0), np.where(m1, f1 - mean - a1, 0.0)
        q0, q1 = np.where(m0, f0 - mean, 0.0), np.where(m1, f1 - mean, 0.0)
        wn = lambda u0, u1: float(np.sqrt(v0 * np.sum(u0 * u0) + v1 * np.sum(u1 * u1)))
        res["solve"]["rel_resid_by_oracle"] = wn(r0, r1) / wn(q0, q1)
        t0 = time.perf_counter()
        try:
            O.amr_solve(flags, nb, p0, p1, f0, f1, pr.rho_neg, pr.rho_pos, rtol=1e-10, max_iter=10)
        except O.OracleError:   # not converged after 10 iterations, as expected
            pass
        per_it = (time.perf_counter() - t0) / 10
        res["solve"]["oracle_ms_per_iter"] = round(per_it * 1e3, 1)
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--nu", type=int, default=2)
    ap.add_argument("--nu-coarse", type=int, default=0,
                    help="sweeps per level below the finest (0: as --nu)")
    ap.add_argument("--methods", default="plain,plain0,plain_d,mixed,mixed0,learned")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--guess-sweeps", type=int, default=2,
                    help="red-black sweeps applied to the learned guess")
    ap.add_argument("--check-every", type=int, default=2,
                    help="CG iterations between host polls of convergence")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--workload", default="rising256",
                    choices=["rising256", "batched64", "single32", "bubbles128",
                             "projection256", "flow256", "heat256", "blocks256", "amr256"],
                    help="rising256: the 256^3 sequence (default); batched64: 64 x 64^3; "
                         "single32 / bubbles128: one fixed problem, plain vs mixed; "
                         "projection256 / flow256: the steps around the solve; heat256: "
                         "implicit heat diffusion; blocks256: block layout; amr256: the "
                         "two-level composite grid (fill, operator, solves)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run a device copy of this many bytes (counter scaling)")
    args = ap.parse_args()
    global NU_COARSE
    NU_COARSE = args.nu_coarse

    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus %d requested); run with --gpus 1" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2312_11740_amd as M
    from paper_2312_11740_amd import problems as G

    if args.copy_calibration:
        copy_calibration(torch, args.copy_calibration)
        return

    dev = torch.device("cuda:0")
    if args.workload == "batched64":
        batched64(M, G, torch, args)
        return
    if args.workload in ("single32", "bubbles128"):
        single_problem(M, G, torch, args, args.workload)
        return
    if args.workload == "projection256":
        projection256(M, G, torch, args)
        return
    if args.workload == "flow256":
        flow256(M, G, torch, args)
        return
    if args.workload == "heat256":
        heat256(M, G, torch, args)
        return
    if args.workload == "blocks256":
        blocks256(M, G, torch, args)
        return
    if args.workload == "amr256":
        amr256(M, G, torch, args)
        return
    n, K, W = args.n, args.steps, args.warmup
    prm = dict(rho_neg=1e-3, rho_pos=1.0, sigma=0.01, rtol=1e-10)
    log("generating %d steps of the %d^3 rising-bubble sequence" % (K + W, n))
    probs = [G.rising_bubble_problem(t, n=n) for t in range(K + W)]
    phis = [torch.from_numpy(q.phi).to(dev) for q in probs]
    fs = [torch.from_numpy(q.f).to(dev) for q in probs]
    ws = torch.empty(M.workspace_bytes(n, 1), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    MODES = {"plain": "fp64", "plain0": "fp64", "plain_d": "fp64", "mixed": "mixed",
             "mixed0": "mixed", "learned": "mixed"}
    DEFLATE = {"plain": False, "plain0": False, "plain_d": True, "mixed": True, "mixed0": True,
               "learned": True}
    ZERO = {"plain0", "mixed0"}
    net = None
    if "learned" in args.methods.split(","):
        net = M.Net(64, 1, device=dev)
        net.load(M.TRAINED_WEIGHTS)
    # untimed burn-in: the first solves after start-up run at lower clocks, which would
    # otherwise bias whichever method is timed first
    run_sequence(M, torch, ws, phis, fs, prm, "fp64", args.nu, min(len(phis), 3), 0, None,
                 zero=True)
    results = {}
    for meth in args.methods.split(","):
        mode = MODES[meth]
        ms, infos, fb = run_sequence(M, torch, ws, phis, fs, prm, mode, args.nu, K, W,
                                     net if meth == "learned" else None, zero=meth in ZERO,
                                     guess_sweeps=args.guess_sweeps,
                                     check_every=args.check_every, deflate=DEFLATE[meth])
        worst = max(i.rel_resid for i in infos)
        ok = all(i.status == M.OK for i in infos) and worst <= prm["rtol"]
        results[meth] = dict(ms=ms, iters=[i.iters for i in infos],
                             outer=[i.outer_iters for i in infos], max_rel_resid=worst, ok=ok,
                             fallbacks=fb)
        log("%s: %.2f ms/step iters %s max rel resid %.2e ok=%s"
            % (meth, ms, results[meth]["iters"], worst, ok))

    # the headline method is learned + mixed; without it, the faster converged one
    best = "learned" if "learned" in results else None
    if best is None:
        best = min((m for m in results if results[m]["ok"]), key=lambda m: results[m]["ms"],
                   default=None)
    if best is None:
        best = min(results, key=lambda m: results[m]["ms"])
    plain_ms = results.get("plain", {}).get("ms")

    roofline = None
    kernels = None
    if not args.no_profile:
        mode = MODES[best]
        stats = run_profiled(M, torch, ws, phis, fs, prm, mode, args.nu, K, W,
                             net if best == "learned" else None, zero=best in ZERO,
                             deflate=DEFLATE[best])
        kernels = {k: dict(launches=v["launches"], mean_us=1e3 * v["ms"] / v["launches"],
                           GBps=(v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["bytes"] else None,
                           share=None)
                   for k, v in stats.items()}
        total = sum(v["ms"] for v in stats.values())
        for k in kernels:
            kernels[k]["share"] = round(stats[k]["ms"] / total, 3)
        dom = max((k for k in stats if stats[k]["bytes"] > 0), key=lambda k: stats[k]["ms"])
        v = stats[dom]
        per_launch = v["bytes"] / v["launches"]
        achieved = per_launch / (v["ms"] * 1e-3 / v["launches"]) / 1e9
        kname = "%s/%s" % (dom, "f64" if MODES[best] == "fp64" else "f32")
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(kname), "kernel": kname,
                    "alg_bytes_per_launch": per_launch,
                    "mean_launch_us": round(1e3 * v["ms"] / v["launches"], 2)}
        log("kernels:", json.dumps(kernels))

    cpu = None
    err = None
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on step 0 (full size)")
        op = M.Operator(phis[0], prm["rho_neg"], prm["rho_pos"], prm["sigma"], workspace=ws)
        g0 = None
        if best == "learned":
            g0, _ = op.learned_guess(net, fs[0], sweeps=2,
                                     judge="deflated" if DEFLATE[best] else "plain")
        p0, _ = op.solve(fs[0], p=g0, rtol=prm["rtol"], mode=MODES[best], nu=args.nu,
                         deflate=DEFLATE[best])
        p0h = p0.cpu().numpy()
        op.close()
        cpu, err, rr = cpu_baseline(probs[0], p0h)
        log("cpu baseline %s, gpu err vs oracle %.3e, oracle-computed residual %.3e"
            % (cpu, err, rr))

    value = results[best]["ms"]
    line = {
        "metric": "time to 1e-10 rel. residual, 256^3 rho-ratio 1000 (learned+mixed vs plain); "
                  "HBM GB/s",
        "value": round(value, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(value, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"plain": "f64", "plain0": "f64", "plain_d": "f64", "mixed": "f32+f64",
                  "mixed0": "f32+f64", "learned": "bf16+f32+f64"}[best],
        "data": "synthetic",
        "config": {"workload": "rising bubble %d^3, density ratio 1000, sigma 0.01, one "
                               "projection solve (operator build + MG-PCG to 1e-10, warm "
                               "start) per step" % n,
                   "n": n, "method": best, "nu": args.nu,
                   "learned_guess": ("U-Net at 64^3 on 4^3-block means, weights "
                                     "paper_2312_11740_amd/weights/unet64.f32"
                                     if best == "learned" else None)},
        "methods": {m: {"ms_per_step": round(r["ms"], 3), "iters": r["iters"],
                        "outer": r["outer"], "max_rel_resid": r["max_rel_resid"],
                        "ok": r["ok"], "guess_fallbacks": r["fallbacks"],
                        "deflated": DEFLATE[m]}
                    for m, r in results.items()},
        "speedup_vs_plain_fp64": (round(plain_ms / value, 3) if plain_ms else None),
        "speedup_vs_best_plain": (round(min(results[m]["ms"] for m in ("plain", "plain0")
                                            if m in results) / value, 3)
                                  if ("plain" in results or "plain0" in results) else None),
        "err_vs_oracle_step0": err,
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
