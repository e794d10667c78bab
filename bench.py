#!/usr/bin/env python3
"""EOFA solve benchmark on one MI355X.

Workload (default): 16^3 x 32 lattice, Ls = 16, Mobius b5 = 1.5, c5 = 0.5,
M5 = 1.8, antiperiodic time; links exp(i 0.5 H) (seeded), one Gaussian
source; the shifted EOFA system of the action and force,
(H(m2) - Delta_+(m1, m2) P_+) psi = phi with m1 = 0.04, m2 = 1.0, solved to
an FP64 true residual of 1e-10 with FP16-storage / FP32-arithmetic inner CG
and an FP64 defect-correction outer loop whose passes keep the inner search
direction (reliable updates; the plain restarted variant is timed beside it
and reported as restarted_defect_correction). A step is one complete solve
(pack, Schur source, outer/inner CG, reconstruction, FP64 true residual,
unpack), inputs resident in HBM.

Output: one JSON line. ``value`` is the whole-job Dslash throughput: the
hop's compulsory bytes (input and output spinor once, links once) of every
inner-solve hop launch divided by the wall time of the timed steps.
``roofline`` is the dominant hop kernel alone on the same bytes (HIP events on
the solve's stream, every 8th iteration), with the fused bytes of its
epilogue and every role's figures beside it. ``dslash_beyond_mall`` times the
single-RHS Dslash on 24^3 x 64 x Ls=12, whose fields exceed the 256 MB MALL.
``cpu_baseline`` times the CPU oracle (plain numpy FP64) on this host: its
off-parity operator on the same lattice, and its solve of the same system on
4^4 x Ls=8 to 1e-10 (the GPU's time on that solve is gpu_c1_time_to_solution).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Dslash HBM GB/s (% peak); EOFA CG time-to-1e-10 residual, mixed/learned vs plain FP64"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: dims (Lx, Ly, Lz, Lt), Ls, eps, m1, gauge seed, source seed
    "c1": ((4, 4, 4, 4), 8, 0.3, 0.04, 1000, 2000),
    "c2": ((16, 16, 16, 32), 16, 0.5, 0.04, 1001, 2001),
}
ROLE_NAMES = ["K1 D~.Mee^-1.Dhop.D~", "K2 Mee.p - Dhop.(D~t)", "K3 Mee^-T.D~^T.Dhop^dag", "K4 r -= a(Mee^T.w - D~^T.Dhop^dag)"]
PREC = {"fp64": 0, "fp32": 1, "fp16s": 2}


def site_bytes(prec):
    """bytes of one 5D site-spinor in a packed field (FP16S: values + scale)."""
    return {0: 192, 1: 96, 2: 52}[prec]


def link_bytes_per_site(prec):
    """8 links x 9 complex per 4D site, in the storage precision."""
    return 72 * {0: 16, 1: 8, 2: 4}[prec]


def role_bytes(role, prec, Ls, Nh):
    """Fused compulsory bytes of one launch of an inner hop kernel: every field
    it touches read once (K2 also reads the same-site p, K4 also reads w and
    reads and writes the residual), every output written once, every link once."""
    E = site_bytes(prec)  # the inner residual is kept in the inner precision too
    lk = link_bytes_per_site(prec) / Ls
    per = {0: 2 * E, 1: 3 * E, 2: 2 * E, 3: 4 * E}[role] + lk
    return per * Nh


def hop_bytes(prec, Ls, Nh):
    """Compulsory bytes of the hop itself, Dhop.D~ on one half-field: the input
    spinor read once, the output written once, the links once per launch
    (FP16S at Ls = 16: 52 + 52 + 288/16 = 122 B per 5D site)."""
    return (2 * site_bytes(prec) + link_bytes_per_site(prec) / Ls) * Nh


def cpu_info():
    """Host core count and CPU model of the machine the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return dict(nproc=os.cpu_count(), usable_cores=usable, cpu_model=model)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1706_05843_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile(workload, prec_name, role):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}_{prec_name}.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch", {}).get(str(role))


def _timed(fn):
    """(result, wall seconds, threads used = process CPU time / wall time)."""
    w0, c0 = time.perf_counter(), time.process_time()
    out = fn()
    w, c = time.perf_counter() - w0, time.process_time() - c0
    return out, w, max(1, int(round(c / max(w, 1e-9))))


def cpu_baseline(dims, Ls, eps, m1, gseed, sseed, plain_iters=None):
    """The CPU oracle as it stands (plain numpy FP64), on this host:
    (1) its off-parity operator Dhop.D~(m) once on the same lattice as the GPU
    step, in the GPU roofline's bytes (the value); (2) its whole solve route
    (mirror mode: Schur source, CGNR, reconstruction) of the same shifted
    system to a 1e-10 residual on the small 4^4 x Ls=8 workload; (3) for the
    full-size solve, which would take hours on the host, an extrapolation:
    four such applications per CGNR iteration (two of the Schur operator, two
    of its adjoint; the same-parity blocks and the vector updates left out,
    so a lower bound) times the GPU's plain FP64 iteration count."""
    import numpy as np
    from oracle import eo
    from oracle.dwf import Action, Dtilde_op, System
    from oracle.lattice import hop, restrict
    from paper_1706_05843_amd import synth
    info = cpu_info()
    act = Action(dims, Ls, 1.8, 1.5, 0.5, (1, 1, 1, -1))
    U = synth.gauge_field(dims, eps, gseed)
    psi = synth.fermion(dims, Ls, sseed)
    x = restrict(psi, dims, 1)
    y, dt, threads = _timed(lambda: restrict(hop(U, Dtilde_op(act, 1.0, x), act.bc), dims, 0))
    del y
    Vh = int(np.prod(dims)) // 2
    byts = hop_bytes(0, Ls, Vh * Ls)
    d1, l1, e1, ms1, gs1, ss1 = WORKLOADS["c1"]
    act1 = Action(d1, l1, 1.8, 1.5, 0.5, (1, 1, 1, -1))
    U1, phi1 = synth.gauge_field(d1, e1, gs1), synth.fermion(d1, l1, ss1)
    out, t1, th1 = _timed(lambda: eo.solve_mirror(act1, U1, System(1.0, ms1, 1.0, -1.0, +1), phi1, tol=1e-10))
    extra = {}
    if plain_iters:
        extra["time_to_solution_extrapolated"] = dict(
            seconds_lower_bound=round(4 * dt * plain_iters, 1), iters=plain_iters,
            basis=f"4 x {dt:.2f} s (measured Dhop.D~ application) x {plain_iters} CGNR iterations "
                  f"(the GPU's plain FP64 count); same-parity blocks and vector updates not counted")
    return dict(value=byts / dt / 1e9, unit="GB/s", cores=threads, kind="oracle",
                sample=f"one application of the oracle's FP64 off-parity operator Dhop.D~ on the full "
                       f"{dims[0]}x{dims[1]}x{dims[2]}x{dims[3]} x Ls={Ls} lattice ({dt:.2f} s), bytes counted "
                       f"like the GPU roofline (input and output spinor once, links once); plus the oracle's "
                       f"solve of H(m2)-Delta_+(m1,m2)P_+ to a 1e-10 residual on 4^4 x Ls=8",
                nproc=info["nproc"], usable_cores=info["usable_cores"], cpu_model=info["cpu_model"],
                time_to_solution_c1=dict(seconds=round(t1, 3), iters=out["iters"], true_resid=out["true_resid"],
                                         cores=th1, workload="4x4x4x4 Ls=8 eps=0.3 m1=0.04 m2=1.0, "
                                         "H(m2)-Delta_+(m1,m2)P_+, CGNR to 1e-10 (mirror mode)"), **extra)


def gpu_c1(eofa, synth, torch):
    """The same 4^4 x Ls=8 solve as the CPU oracle's time-to-solution, on the GPU."""
    d1, l1, e1, ms1, gs1, ss1 = WORKLOADS["c1"]
    U = torch.from_numpy(synth.gauge_field(d1, e1, gs1)).cuda()
    phi = torch.from_numpy(synth.fermion(d1, l1, ss1, nrhs=1)).cuda()
    psi = torch.zeros_like(phi)
    ctx = eofa.Context(eofa.make_action(d1, l1, 1.8, 1.5, 0.5), U)
    res = {}
    for name, prec in (("fp64", eofa.FP64), ("fp16s", eofa.FP16S)):
        prm = eofa.make_params(tol=1e-10, inner_prec=prec)
        ctx.eofa_cg_solve([(1.0, ms1, 1.0, -1.0, +1)], phi, psi, prm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, st = ctx.eofa_cg_solve([(1.0, ms1, 1.0, -1.0, +1)], phi, psi, prm)
        torch.cuda.synchronize()
        res[name] = dict(seconds=round(time.perf_counter() - t0, 5), iters=st[0]["iters"],
                         true_resid=st[0]["true_resid"], rc=rc)
    ctx.close()
    return res


def dslash_beyond_mall(eofa, synth, torch, np, reps=100):
    """Single-RHS Dslash (Dhop.D~, odd -> even) on the 24^3 x 64 x Ls=12
    lattice, whose FP16S half-field (263 MiB) and FP32/FP64 ones exceed the
    256 MB MALL, so every launch streams from HBM. Algorithmic GB/s on the hop's
    compulsory bytes, HIP events on the launch stream over `reps` launches."""
    dims, Ls, eps, m1 = (24, 24, 24, 64), 12, 0.5, 0.01
    U = torch.from_numpy(synth.gauge_field(dims, eps, 1003)).cuda()
    ctx = eofa.Context(eofa.make_action(dims, Ls, 1.8, 1.5, 0.5), U)
    del U
    phi = synth.fermion_torch(dims, Ls, seed=2003, nrhs=1)
    Nh = int(np.prod(dims)) // 2 * Ls
    out = {}
    sysl = [(m1, m1, 1.0, 0.0, -1)]
    for name, prec in (("fp16s", eofa.FP16S), ("fp32", eofa.FP32), ("fp64", eofa.FP64)):
        pin, pout = ctx.new_packed(prec, 1), ctx.new_packed(prec, 1)
        ctx.eofa_pack(phi, pin, 1, prec, 1)
        ctx.eofa_dslash(sysl, pin, pout, 0, 0, prec, 1)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(reps):
            ctx.eofa_dslash(sysl, pin, pout, 0, 0, prec, 1)
        ev[1].record()
        torch.cuda.synchronize()
        t = ev[0].elapsed_time(ev[1]) / reps * 1e-3
        gbs = hop_bytes(prec, Ls, Nh) / t / 1e9
        out[name] = dict(avg_launch_us=round(t * 1e6, 2), algorithmic_GBs=round(gbs, 1),
                         frac_hbm=round(gbs / HBM_PEAK_GBS, 4), gflops=round(1320.0 * Nh / t / 1e9, 1),
                         field_MiB=round(ctx.packed_bytes(prec, 1) / 2 ** 20, 1),
                         bytes_per_launch=int(hop_bytes(prec, Ls, Nh)))
        del pin, pout
    ctx.close()
    return dict(workload=f"{dims[0]}x{dims[1]}x{dims[2]}x{dims[3]} Ls={Ls}, one Gaussian RHS, Dhop.D~(m1={m1}) "
                         f"odd->even, {reps} launches", **out)


def bench_batched(args, eofa, synth, torch, np):
    """Batched multi-right-hand-side workload: 24^3 x 64, Ls = 12, m1 = 0.01,
    12 Gaussian right-hand sides (6 on H(m1), 6 on H(m2) - Delta_+(m1,m2) P_+),
    FP32 inner / FP64 outer. Times (a) one 12-RHS Dslash launch against 12
    single-RHS launches, (b) a fixed number of batched inner CG iterations
    (HIP graph, autotuned launch shape) against 12 single-RHS solves."""
    dims, Ls, eps, m1, m2, nrhs = (24, 24, 24, 64), 12, 0.5, 0.01, 1.0, 12
    print(f"bench: batched workload dims={dims} Ls={Ls} nrhs={nrhs}", file=sys.stderr, flush=True)
    U = torch.from_numpy(synth.gauge_field(dims, eps, 1003)).cuda()
    ctx = eofa.Context(eofa.make_action(dims, Ls, 1.8, 1.5, 0.5), U)
    phi = synth.fermion_torch(dims, Ls, seed=2003, nrhs=nrhs)
    Vh = int(np.prod(dims)) // 2
    Nh = Vh * Ls
    prec = eofa.FP32
    sysl = [(m1, m1, m2, 0.0, -1)] * (nrhs // 2) + [(m2, m1, m2, -1.0, +1)] * (nrhs - nrhs // 2)
    # autotune the launch shape on a short batched solve first; the Dslash
    # entry point then uses the same tuned shape
    iters = args.batched_iters
    psi = torch.zeros_like(phi)
    prm = eofa.make_params(fixed_iters=iters, inner_prec=prec, use_graph=1, check_every=16)
    _, st = ctx.eofa_cg_solve(sysl, phi, psi, prm)
    tuned = (st[0]["waves"], st[0]["rhs_block"])
    # (a) Dslash: one launch over all right-hand sides vs one launch each
    pin, pout = ctx.new_packed(prec, nrhs), ctx.new_packed(prec, nrhs)
    ctx.eofa_pack(phi, pin, 1, prec, nrhs)
    reps = 100
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ctx.eofa_dslash(sysl, pin, pout, 0, 0, prec, nrhs)
    ev[0].record()
    for _ in range(reps):
        ctx.eofa_dslash(sysl, pin, pout, 0, 0, prec, nrhs)
    ev[1].record()
    # single-RHS launches, each on its own right-hand side (FP32 packed fields
    # hold one contiguous block per right-hand side), so no launch finds its
    # input left in the caches by the one before
    b1 = ctx.packed_bytes(prec, 1)
    assert ctx.packed_bytes(prec, nrhs) == nrhs * b1
    ctx.eofa_dslash(sysl[:1], pin[:b1], pout[:b1], 0, 0, prec, 1)
    ev[2].record()
    for _ in range(reps):
        for r in range(nrhs):
            ctx.eofa_dslash(sysl[r:r + 1], pin[r * b1:(r + 1) * b1], pout[r * b1:(r + 1) * b1], 0, 0, prec, 1)
    ev[3].record()
    torch.cuda.synchronize()
    t_multi = ev[0].elapsed_time(ev[1]) / reps * 1e-3
    t_single = ev[2].elapsed_time(ev[3]) / reps * 1e-3
    alg = (2 * site_bytes(prec) * Nh * nrhs + link_bytes_per_site(prec) * Vh)
    alg1 = (2 * site_bytes(prec) * Nh + link_bytes_per_site(prec) * Vh) * nrhs
    del pin, pout
    # (b) batched inner iterations
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rc, st = ctx.eofa_cg_solve(sysl, phi, psi, prm)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.steps
    ph1, ps1 = phi[:1].clone(), torch.zeros_like(phi[:1])
    ctx.eofa_cg_solve(sysl[:1], ph1, ps1, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(nrhs):
        ph1.copy_(phi[r:r + 1])
        ctx.eofa_cg_solve(sysl[r:r + 1], ph1, ps1, prm)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    # (c) time to solution: the 12 systems to an FP64 true residual of 1e-10,
    # batched (FP32 inner, HIP graph, autotuned shape) against 12 plain FP64 solves
    conv = None
    if not args.no_converge:
        prm_c = eofa.make_params(tol=1e-10, inner_prec=prec, use_graph=1, check_every=16)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, st = ctx.eofa_cg_solve(sysl, phi, psi, prm_c)
        torch.cuda.synchronize()
        t_conv = time.perf_counter() - t0
        its = [s["iters"] for s in st]
        conv = dict(seconds=round(t_conv, 3), rc=rc, iters=its, max_true_resid=max(s["true_resid"] for s in st),
                    all_converged=all(s["converged"] for s in st),
                    per_rhs_iteration_ms=round(t_conv / sum(its) * 1e3, 4),
                    ideal_per_rhs_iteration_ms_fp32=round(17 * site_bytes(1) * Nh / HBM_PEAK_GBS / 1e6
                                                           + 4 * link_bytes_per_site(1) * Vh / HBM_PEAK_GBS / 1e6, 4))
        print(f"bench: batched converged solve {conv}", file=sys.stderr, flush=True)
        if not args.no_plain:
            prm_p = eofa.make_params(tol=1e-10, inner_prec=eofa.FP64, check_every=16)
            t0 = time.perf_counter()
            plain = []
            for r in range(nrhs):
                ph1.copy_(phi[r:r + 1])
                rc1, st1 = ctx.eofa_cg_solve(sysl[r:r + 1], ph1, ps1, prm_p)
                plain.append(dict(rc=rc1, iters=st1[0]["iters"], true_resid=st1[0]["true_resid"]))
                print(f"bench: plain FP64 solve {r}: {plain[-1]}", file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            t_plain = time.perf_counter() - t0
            conv["plain_fp64_12_solves_seconds"] = round(t_plain, 3)
            conv["plain_fp64_iters"] = [p_["iters"] for p_ in plain]
            conv["speedup_vs_plain_fp64"] = round(t_plain / t_conv, 3)
    out = {
        "metric": METRIC, "value": round(alg / t_multi / 1e9, 1), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": round(t_batch * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{dims[0]}x{dims[1]}x{dims[2]}x{dims[3]} Ls={Ls} m1={m1} m2={m2}, {nrhs} Gaussian RHS "
                               f"(6 on H(m1), 6 on H(m2)-Delta_+P_+), FP32 inner, {iters} batched CG iterations "
                               f"per step in a HIP graph", "lattice": list(dims), "Ls": Ls, "nrhs": nrhs},
        "dslash_multi_rhs": {"seconds_per_launch": t_multi, "algorithmic_GBs": round(alg / t_multi / 1e9, 1),
                             "frac_hbm": round(alg / t_multi / 1e9 / HBM_PEAK_GBS, 4),
                             "single_rhs_launches_seconds": t_single,
                             "single_rhs_algorithmic_GBs": round(alg1 / t_single / 1e9, 1),
                             "speedup_one_launch_vs_12": round(t_single / t_multi, 3),
                             "tuned_waves_rhs_block": list(tuned)},
        "batched_cg": {"iters": iters, "seconds_batched": t_batch, "seconds_12_single": t_seq,
                       "speedup": round(t_seq / t_batch, 3),
                       "per_rhs_iteration_ms": round(t_batch / nrhs / iters * 1e3, 4)},
        "time_to_solution_1e-10": conv,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_learned(args, eofa, synth, torch, np):
    """Learned preconditioner workload: 16^3 x 32, Ls = 16, eps = 0.5, the
    shifted system H(m2) - Delta_+(m1, m2) P_+ (m1 = 0.04, m2 = 1.0). Training
    pairs (r_k, e_k = x* - x_k) from FP64 CG on the normal equations of
    args.train_fields seeded gauge fields (args.pairs_per_field each, spread
    over the CG run); a network N = B^dag B with B of channels args.channels
    (default 1 -> 4 -> 1) trained with Adam on the GPU; then, on
    args.held_fields held-out fields, time to an FP64 true residual of 1e-10
    for plain FP64 CGNR, FP16S/FP64 mixed CGNR, flexible CG with the
    identity, and flexible CG with the trained network (network in FP32,
    operator in FP64). The loss is the scale-free residual loss
    1 - |<A N(r), r>|^2/(|A N(r)|^2 |r|^2) (A = M^dag M) unless --loss error."""
    dims, Ls, eps, m1, m2 = (16, 16, 16, 32), 16, 0.5, 0.04, 1.0
    system = (m2, m1, m2, -1.0, +1)
    chans = [int(c) for c in args.channels.split(",")]
    act = eofa.make_action(dims, Ls, 1.8, 1.5, 0.5)
    log = lambda m: print(f"bench: {m}", file=sys.stderr, flush=True)
    log(f"learned workload dims={dims} Ls={Ls}, {args.train_fields} training + {args.held_fields} held-out fields")
    ctxs, data = [], []
    t0 = time.perf_counter()
    stride = None
    npf = args.pairs_per_field
    for f in range(args.train_fields):
        ctx = eofa.Context(act, torch.from_numpy(synth.gauge_field(dims, eps, 3000 + f)).cuda())
        phi = synth.fermion_torch(dims, Ls, seed=3100 + f, nrhs=1)
        b = ctx.packed_bytes(eofa.FP32)
        if stride is None:  # spread the pairs over the CG run of the first field
            r1 = torch.empty(b, dtype=torch.uint8, device="cuda")
            _, _, its = ctx.eofa_cg_pairs(system, phi, 1, 0, 1, 1e-12, 50000, r1, r1.clone())
            stride = max(1, its // npf)
            log(f"training CG runs {its} iterations to 1e-12; pair stride {stride}")
        r = torch.empty(npf * b, dtype=torch.uint8, device="cuda")
        e = torch.empty(npf * b, dtype=torch.uint8, device="cuda")
        rc, rec, its = ctx.eofa_cg_pairs(system, phi, npf, 0, stride, 1e-12, 50000, r, e)
        ctxs.append(ctx)
        data.append((r, e, rec))
        log(f"field {f}: {rec} pairs, CG {its} iterations")
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    npairs = sum(d[2] for d in data)
    net = eofa.Net(ctxs[0], chans, seed=7, init_scale=0.25)
    # loss of the untrained network
    lsys = system if args.loss == "residual" else None
    loss0 = sum(net.loss_grad(c, d[0], d[1], d[2], system=lsys)[0] for c, d in zip(ctxs, data)) / npairs
    t0 = time.perf_counter()
    hist = []
    for ep in range(args.epochs):
        tot = 0.0
        for c, (r, e, rec) in zip(ctxs, data):
            tot += net.train(c, r, e, rec, epochs=1, batch=args.batch, lr=args.lr, system=lsys)[0] * rec
        hist.append(tot / npairs)
        log(f"epoch {ep}: mean loss per pair {hist[-1]:.4f}")
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    for c in ctxs:
        c.close()
    del data
    torch.cuda.empty_cache()

    def timed(ctx, phi, prm):
        psi = torch.zeros_like(phi)
        torch.cuda.synchronize()
        t = time.perf_counter()
        rc, st = ctx.eofa_cg_solve([system], phi, psi, prm)
        torch.cuda.synchronize()
        return dict(seconds=time.perf_counter() - t, iters=st[0]["iters"], true_resid=st[0]["true_resid"],
                    converged=st[0]["converged"], fell_back=st[0]["fell_back"], rc=rc)

    modes = {
        "plain_fp64": eofa.make_params(tol=1e-10, inner_prec=eofa.FP64),
        "mixed_fp16s": eofa.make_params(tol=1e-10, inner_prec=eofa.FP16S, keep_direction=1),
        "fgcg_identity": eofa.make_params(tol=1e-10, precond=1),
        "fgcg_learned": eofa.make_params(tol=1e-10, precond=1, net=net),
        "fgcg_learned_window8": eofa.make_params(tol=1e-10, precond=1, net=net, fcg_window=8),
    }
    res = {k: [] for k in modes}
    t_apply = None
    for f in range(args.held_fields):
        ctx = eofa.Context(act, torch.from_numpy(synth.gauge_field(dims, eps, 4000 + f)).cuda())
        phi = synth.fermion_torch(dims, Ls, seed=4100 + f, nrhs=1)
        if f == 0:
            for prm in modes.values():  # warm-up (autotune, workspace)
                timed(ctx, phi, prm)
            # one application of N (B and B^dag, all layers) on the default stream
            pin, pout = ctx.new_packed(eofa.FP32), ctx.new_packed(eofa.FP32)
            pin.zero_()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            net.apply(ctx, pin, pout)
            ev0.record()
            for _ in range(10):
                net.apply(ctx, pin, pout)
            ev1.record()
            torch.cuda.synchronize()
            t_apply = ev0.elapsed_time(ev1) / 10 * 1e-3
        for k, prm in modes.items():
            res[k].append(timed(ctx, phi, prm))
        log(f"held-out field {f}: " + ", ".join(f"{k} {v[-1]['iters']} it {v[-1]['seconds']:.3f} s" for k, v in res.items()))
        ctx.close()
    summ = {}
    for k, v in res.items():
        summ[k] = dict(mean_seconds=round(float(np.mean([x["seconds"] for x in v])), 5),
                       mean_iters=round(float(np.mean([x["iters"] for x in v])), 1),
                       max_true_resid=float(max(x["true_resid"] for x in v)),
                       all_converged=all(x["converged"] == 1 for x in v),
                       fell_back=sum(x["fell_back"] for x in v))
    plain = summ["plain_fp64"]["mean_seconds"]
    out = {
        "metric": METRIC, "value": summ["fgcg_learned"]["mean_seconds"], "unit": "s", "n_gpus": 1,
        "steps": args.held_fields, "warmup": 1, "ms_per_step": round(summ["fgcg_learned"]["mean_seconds"] * 1e3, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{dims[0]}x{dims[1]}x{dims[2]}x{dims[3]} Ls={Ls}, system H(m2)-Delta_+(m1,m2)P_+ "
                               f"m1={m1} m2={m2}; network {chans}, bfloat16 weights, FP32 arithmetic; "
                               f"{npairs} training pairs from {args.train_fields} fields, {args.epochs} epochs; "
                               f"FGCG to true residual 1e-10 on {args.held_fields} held-out fields",
                   "lattice": list(dims), "Ls": Ls},
        "modes": summ,
        "time_ratio_vs_plain_fp64": {k: round(v["mean_seconds"] / plain, 3) for k, v in summ.items()},
        "iteration_ratio_learned_vs_identity": round(summ["fgcg_learned"]["mean_iters"] /
                                                     summ["fgcg_identity"]["mean_iters"], 3),
        "network_apply_ms": None if t_apply is None else round(t_apply * 1e3, 3),
        "training": {"pairs": npairs, "pair_stride": stride, "seconds_pairs": round(t_pairs, 2),
                     "seconds_training": round(t_train, 2), "loss_untrained": loss0, "loss_per_epoch": hist,
                     "epochs": args.epochs, "batch": args.batch, "lr": args.lr, "loss": args.loss},
    }
    net.close()
    print(json.dumps(out), flush=True)


def bench_force(args, eofa, synth, torch, np):
    """EOFA pseudofermion force (eqn eofa_force) on 16^3 x 32, Ls = 16: the two
    solves chi_1, chi_2 as one batched FP16S/FP64 solve to 1e-10, then the link
    derivative kernels. Reports the whole force time and the link-derivative
    kernel alone (HIP events on the stream it runs on) against its compulsory
    bytes: chi read once (V Ls 192 B), links read and force written once
    (4 V 144 B each)."""
    dims, Ls, eps, m1, m2 = (16, 16, 16, 32), 16, 0.5, 0.04, 1.0
    U = torch.from_numpy(synth.gauge_field(dims, eps, 1001)).cuda()
    ctx = eofa.Context(eofa.make_action(dims, Ls, 1.8, 1.5, 0.5), U)
    phi = torch.from_numpy(synth.fermion(dims, Ls, 2001, nrhs=1)).cuda()
    F = torch.zeros(ctx.gauge_shape(), dtype=torch.complex128, device="cuda")
    prm = eofa.make_params(tol=1e-10, inner_prec=eofa.FP16S)
    ctx.eofa_force(m1, m2, phi, F, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rc, st = ctx.eofa_force(m1, m2, phi, F, prm)
    torch.cuda.synchronize()
    t_force = (time.perf_counter() - t0) / args.steps
    y = torch.zeros_like(F)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ctx.eofa_dhop_derivative(phi, phi, y)
    reps = 100
    ev[0].record()
    for _ in range(reps):
        ctx.eofa_dhop_derivative(phi, phi, y)
    ev[1].record()
    torch.cuda.synchronize()
    t_k = ev[0].elapsed_time(ev[1]) / reps * 1e-3
    V = int(np.prod(dims))
    alg = V * Ls * 192 + 2 * 4 * V * 144
    out = {
        "metric": METRIC, "value": round(t_force, 5), "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": round(t_force * 1e3, 3), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{dims[0]}x{dims[1]}x{dims[2]}x{dims[3]} Ls={Ls}, EOFA force m1={m1} m2={m2}, "
                               f"chi_1, chi_2 by one batched FP16S/FP64 solve to 1e-10", "lattice": list(dims),
                   "Ls": Ls},
        "solves": [dict(iters=x["iters"], true_resid=x["true_resid"]) for x in st],
        "link_derivative_kernel": {"seconds": t_k, "algorithmic_bytes": alg,
                                   "algorithmic_GBs": round(alg / t_k / 1e9, 1),
                                   "frac_hbm": round(alg / t_k / 1e9 / HBM_PEAK_GBS, 4)},
    }
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_heatbath(args, eofa, synth, torch, np):
    """EOFA heatbath (eqn eofa_heatbath) on 16^3 x 32, Ls = 16 with a 6-pole
    partial-fraction approximation of x^-1/2 (6-node Gauss-Legendre rule for
    x^-1/2 = (2/pi) int_0^1 du / (u^2 + x (1 - u)^2), written as
    sum_l alpha_l / (beta_l + x); 1e-4 relative on [0.5, 4]).
    Modes (Sec. VI B): all 12 systems in one batched solve; poles one after
    another from chronological forecasts; forecasts plus per-pole tolerances
    relaxed by each pole's weight k alpha_l gamma_l^2 in phi. Inner FP16S,
    outer FP64."""
    dims, Ls, eps, m1, m2 = (16, 16, 16, 32), 16, 0.5, 0.04, 1.0
    U = torch.from_numpy(synth.gauge_field(dims, eps, 1001)).cuda()
    ctx = eofa.Context(eofa.make_action(dims, Ls, 1.8, 1.5, 0.5), U)
    eta = torch.from_numpy(synth.fermion(dims, Ls, 2002, nrhs=1)).cuda()
    # (2/pi) int_0^1 du / ((1 - u)^2 (x + u^2 / (1 - u)^2)) on a 6-node Gauss-Legendre rule
    uu, ww = np.polynomial.legendre.leggauss(6)
    uu, ww = 0.5 * (uu + 1.0), 0.5 * ww
    beta = [float(x * x / (1.0 - x) ** 2) for x in uu]
    alpha = [0.0] + [float(2.0 / np.pi * wk / (1.0 - x) ** 2) for x, wk in zip(uu, ww)]
    c, d = 1.0, 0.5  # (b5 + c5)/2, (b5 - c5)/2
    Nf = lambda m: (c + d) ** Ls + m * (c - d) ** Ls
    k = 2.0 * c * (m2 - m1) * (c + d) ** (2 * Ls) / (Nf(m1) * Nf(m2))
    wts = [abs(a) * k / (1.0 + b) ** 2 for a, b in zip(alpha[1:], beta)]
    tol = 1e-10
    ptol = [float(min(1e-5, tol * max(wts) / wl)) for wl in wts] * 2
    res = {}
    ref = None
    kd = dict(inner_prec=eofa.FP16S)  # restarted passes: kept directions do not pay off here
    for name, prm, pt in [("batched", eofa.make_params(tol=tol, **kd), None),
                          ("forecast", eofa.make_params(tol=tol, use_guess=1, **kd), None),
                          ("forecast_pole_tol", eofa.make_params(tol=tol, use_guess=1, **kd), ptol)]:
        phi = torch.zeros_like(eta)
        ctx.eofa_heatbath_solve(m1, m2, alpha, beta, eta, phi, prm, pole_tol=pt)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, st = ctx.eofa_heatbath_solve(m1, m2, alpha, beta, eta, phi, prm, pole_tol=pt)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if ref is None:
            ref = phi.clone()
        diff = float(torch.linalg.vector_norm(phi - ref) / torch.linalg.vector_norm(ref))
        res[name] = dict(seconds=round(dt, 4), iters=[s["iters"] for s in st], total_iters=sum(s["iters"] for s in st),
                         rel_diff_vs_batched=diff, rc=rc)
        print(f"bench: heatbath {name}: {dt:.3f} s, iterations {res[name]['iters']}", file=sys.stderr, flush=True)
    out = {
        "metric": METRIC, "value": res["forecast_pole_tol"]["seconds"], "unit": "s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": round(res["forecast_pole_tol"]["seconds"] * 1e3, 3), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{dims[0]}x{dims[1]}x{dims[2]}x{dims[3]} Ls={Ls}, EOFA heatbath m1={m1} m2={m2}, "
                               f"6 poles (12 systems), FP16S inner / FP64 outer, tol {tol}", "lattice": list(dims),
                   "Ls": Ls},
        "poles": {"alpha": alpha, "beta": beta, "pole_tol": ptol},
        "modes": res,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_gparity(args, eofa, synth, torch, np):
    """G-parity in x on 32^3 x 64, Ls = 12 (two flavours: the library holds the
    x-doubled 64 x 32 x 32 x 64 lattice): a 4-RHS FP32 Dslash launch (fields far
    larger than the 256 MB MALL, so this is HBM-bound territory) against its
    compulsory bytes, and one FP16S/FP64 solve of H(m2) - Delta_+(m1,m2) P_+ to
    1e-10 (m1 = 0.0025, m2 = 1.0)."""
    dims, Ls, eps, m1, m2 = (32, 32, 32, 64), 12, 0.5, 0.0025, 1.0
    log = lambda m: print(f"bench: {m}", file=sys.stderr, flush=True)
    log("G-parity workload: generating the 32^3x64 gauge field")
    U = torch.from_numpy(synth.gauge_field(dims, eps, 1005)).cuda()
    act = eofa.make_action(dims, Ls, 1.8, 1.5, 0.5, bc=(2, 1, 1, -1))
    ctx = eofa.Context(act, U)
    del U
    torch.cuda.empty_cache()
    Vd = 2 * int(np.prod(dims))  # doubled lattice
    Nh = Vd // 2 * Ls
    nrhs = 4
    prec = eofa.FP32
    sysl = [(m1, 0.0, 0.0, 0.0, 1)] * nrhs
    src = synth.fermion_torch((2 * dims[0],) + dims[1:], Ls, seed=2005, nrhs=nrhs)
    pin, pout = ctx.new_packed(prec, nrhs), ctx.new_packed(prec, nrhs)
    ctx.eofa_pack(src, pin, 1, prec, nrhs)
    del src
    torch.cuda.empty_cache()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ctx.eofa_dslash(sysl, pin, pout, 0, 0, prec, nrhs)
    reps = 100
    ev[0].record()
    for _ in range(reps):
        ctx.eofa_dslash(sysl, pin, pout, 0, 0, prec, nrhs)
    ev[1].record()
    torch.cuda.synchronize()
    t_d = ev[0].elapsed_time(ev[1]) / reps * 1e-3
    alg = 2 * site_bytes(prec) * Nh * nrhs + link_bytes_per_site(prec) * (Vd // 2)
    log(f"4-RHS Dslash {t_d * 1e3:.2f} ms, {alg / t_d / 1e9:.1f} GB/s")
    del pin, pout
    torch.cuda.empty_cache()
    phi = synth.fermion_torch((2 * dims[0],) + dims[1:], Ls, seed=2006, nrhs=1)
    psi = torch.zeros_like(phi)
    prm = eofa.make_params(tol=1e-10, inner_prec=eofa.FP16S)
    system = [(m2, m1, m2, -1.0, +1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st = ctx.eofa_cg_solve(system, phi, psi, prm)
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t0
    log(f"solve {t_s:.2f} s, {st[0]['iters']} iterations, residual {st[0]['true_resid']:.2e}")
    out = {
        "metric": METRIC, "value": round(alg / t_d / 1e9, 1), "unit": "GB/s", "n_gpus": 1, "steps": reps,
        "warmup": 1, "ms_per_step": round(t_d * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{dims[0]}x{dims[1]}x{dims[2]}x{dims[3]} Ls={Ls}, G-parity in x (2 flavours), "
                               f"4-RHS FP32 Dslash; FP16S/FP64 solve of H(m2)-Delta_+ P_+ m1={m1} m2={m2}",
                   "lattice": list(dims), "Ls": Ls},
        "dslash_4rhs": {"seconds": t_d, "algorithmic_bytes": alg, "algorithmic_GBs": round(alg / t_d / 1e9, 1),
                        "frac_hbm": round(alg / t_d / 1e9 / HBM_PEAK_GBS, 4)},
        "solve": {"seconds": round(t_s, 3), "iters": st[0]["iters"], "outer_iters": st[0]["outer_iters"],
                  "true_resid": st[0]["true_resid"], "rc": rc},
    }
    ctx.close()
    print(json.dumps(out), flush=True)


def inv_sqrt_rational(lmin, lmax, n, np):
    """Coefficients (alpha_0..alpha_n, beta_1..beta_n) of a rational
    approximation alpha_0 + sum alpha_k/(beta_k + x) of x^-1/2 on [lmin, lmax]:
    Gauss-Legendre quadrature of (2/pi) int_0^inf dt/(t^2 + x) with
    t = sqrt(c) tan(theta), c = sqrt(lmin lmax); an input of the heatbath, with
    its largest relative error on the interval."""
    c = np.sqrt(lmin * lmax)
    x, w = np.polynomial.legendre.leggauss(n)
    th, w = 0.25 * np.pi * (x + 1.0), 0.25 * np.pi * w
    beta = c * np.tan(th) ** 2
    alpha = 2.0 * np.sqrt(c) * w / (np.pi * np.cos(th) ** 2)
    xs = np.geomspace(lmin, lmax, 4001)
    f = np.sum(alpha[None, :] / (beta[None, :] + xs[:, None]), axis=1)
    return [0.0] + alpha.tolist(), beta.tolist(), float(np.max(np.abs(1.0 - np.sqrt(xs) * f)))


def bench_c5(args, eofa, synth, torch, np):
    """The G-parity workload end to end: 32^3 x 64, Ls = 12, G-parity in x (the
    library holds the x-doubled 64 x 32 x 32 x 64 lattice), m1 = 0.0025,
    m2 = 1.0. (a) a 4-RHS FP32 Dslash against its compulsory bytes; (b) the
    heatbath phi = f(M_EOFA) eta with 2 poles, its 4 systems in one batched
    solve; (c) the pseudofermion force, its 2 systems (chi_1, chi_2) batched.
    Solves: FP16S inner CG, FP64 defect correction (restarted passes: kept
    directions go stale at this mass), FP64 true residual 1e-10 per system."""
    dims, Ls, eps, m1, m2 = (32, 32, 32, 64), 12, 0.5, 0.0025, 1.0
    log = lambda m: print(f"bench: {m}", file=sys.stderr, flush=True)
    log("C5 workload: generating the 32^3x64 gauge field")
    U = torch.from_numpy(synth.gauge_field(dims, eps, 1005)).cuda()
    act = eofa.make_action(dims, Ls, 1.8, 1.5, 0.5, bc=(2, 1, 1, -1))
    ctx = eofa.Context(act, U)
    del U
    torch.cuda.empty_cache()
    Vd = 2 * int(np.prod(dims))
    Nh = Vd // 2 * Ls
    nrhs, prec = 4, eofa.FP32
    sysl = [(m1, 0.0, 0.0, 0.0, 1)] * nrhs
    src = synth.fermion_torch((2 * dims[0],) + dims[1:], Ls, seed=2005, nrhs=nrhs)
    pin, pout = ctx.new_packed(prec, nrhs), ctx.new_packed(prec, nrhs)
    ctx.eofa_pack(src, pin, 1, prec, nrhs)
    del src
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ctx.eofa_dslash(sysl, pin, pout, 0, 0, prec, nrhs)
    reps = 100
    ev[0].record()
    for _ in range(reps):
        ctx.eofa_dslash(sysl, pin, pout, 0, 0, prec, nrhs)
    ev[1].record()
    torch.cuda.synchronize()
    t_d = ev[0].elapsed_time(ev[1]) / reps * 1e-3
    alg = nrhs * 2 * site_bytes(prec) * Nh + link_bytes_per_site(prec) * (Vd // 2)
    log(f"4-RHS Dslash {t_d * 1e3:.2f} ms, {alg / t_d / 1e9:.1f} GB/s")
    del pin, pout
    torch.cuda.empty_cache()
    eta = synth.fermion_torch((2 * dims[0],) + dims[1:], Ls, seed=2007, nrhs=1)
    phi = torch.zeros_like(eta)
    lo, hi, npol = 0.8, 5.0, 2
    alpha, beta, rat_err = inv_sqrt_rational(lo, hi, npol, np)
    prm = eofa.make_params(tol=1e-10, inner_prec=eofa.FP16S, max_iter=200000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc_h, st_h = ctx.eofa_heatbath_solve(m1, m2, alpha, beta, eta, phi, prm)
    torch.cuda.synchronize()
    t_h = time.perf_counter() - t0
    log(f"heatbath {t_h:.2f} s rc {rc_h}, iterations {[s_['iters'] for s_ in st_h]}")
    force = torch.zeros((4,) + (dims[3], dims[2], dims[1], dims[0], 3, 3), dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc_f, st_f = ctx.eofa_force(m1, m2, phi, force, prm)
    torch.cuda.synchronize()
    t_f = time.perf_counter() - t0
    log(f"force {t_f:.2f} s rc {rc_f}, iterations {[s_['iters'] for s_ in st_f]}")
    out = {
        "metric": METRIC, "value": round(alg / t_d / 1e9, 1), "unit": "GB/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": round((t_h + t_f) * 1e3, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{dims[0]}x{dims[1]}x{dims[2]}x{dims[3]} Ls={Ls}, G-parity in x, m1={m1} m2={m2}: "
                               f"heatbath ({npol} poles, {2 * npol} systems batched) and force (2 systems batched), "
                               f"FP16S inner / FP64 outer, 1e-10 per system; 4-RHS FP32 Dslash",
                   "lattice": list(dims), "Ls": Ls},
        "dslash_4rhs": {"seconds": t_d, "algorithmic_bytes": alg, "algorithmic_GBs": round(alg / t_d / 1e9, 1),
                        "frac_hbm": round(alg / t_d / 1e9 / HBM_PEAK_GBS, 4)},
        "heatbath": {"seconds": round(t_h, 3), "rc": rc_h, "iters": [s_["iters"] for s_ in st_h],
                     "true_resid": [s_["true_resid"] for s_ in st_h], "rational_interval": [lo, hi],
                     "rational_max_rel_error": rat_err, "n_poles": npol},
        "force": {"seconds": round(t_f, 3), "rc": rc_f, "iters": [s_["iters"] for s_ in st_f],
                  "true_resid": [s_["true_resid"] for s_ in st_f]},
        "time_to_solution_s": round(t_h + t_f, 3),
    }
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_dense(args, eofa, synth, torch, np):
    """The paper's Cayley form (App. B.2: D~^-1 right preconditioning, sparse
    fifth-dimension blocks) against the dense form of the same EOFA system
    (off-parity Dhop, same-parity D_ee = M_ee D~^-1 dense in s) on the default
    16^3 x 32, Ls = 16 workload, both to an FP64 true residual of 1e-10, with
    FP64 and FP16S inner CG. Per form: time, iterations, per-kernel average
    launch time and algorithmic GB/s (both forms move the same bytes: the
    Ls x Ls matrices are staged in LDS once per work-group)."""
    dims, Ls, eps, m1, gseed, sseed = WORKLOADS["c2"]
    m2 = 1.0
    log = lambda m: print(f"bench: {m}", file=sys.stderr, flush=True)
    U = torch.from_numpy(synth.gauge_field(dims, eps, gseed)).cuda()
    phi = torch.from_numpy(synth.fermion(dims, Ls, sseed, nrhs=1)).cuda()
    psi = torch.zeros_like(phi)
    ctx = eofa.Context(eofa.make_action(dims, Ls, 1.8, 1.5, 0.5), U)
    system = [(m2, m1, m2, -1.0, +1)]
    Nh = int(np.prod(dims)) // 2 * Ls
    res = {}
    for pname in ("fp64", "fp16s"):
        prec = PREC[pname]
        for form, fname in ((0, "cayley"), (1, "dense")):
            prm = eofa.make_params(tol=1e-10, inner_prec=prec, profile=1, form=form, keep_direction=1)
            ctx.eofa_cg_solve(system, phi, psi, prm)  # warm-up (autotune)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, st = ctx.eofa_cg_solve(system, phi, psi, prm)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            if rc != eofa.EOFA_OK:
                raise RuntimeError(f"{fname} {pname} solve failed rc={rc}")
            s0 = st[0]
            timed = max(s0["hop_timed"], 1)
            us = [h / timed * 1e3 for h in s0["hop_ms"]]
            gbs = [role_bytes(k, prec, Ls, Nh) / (us[k] * 1e-6) / 1e9 for k in range(4)]
            per_iter = sum(role_bytes(k, prec, Ls, Nh) for k in range(4))
            res[f"{fname}_{pname}"] = dict(seconds=round(t, 4), iters=s0["iters"], outer_iters=s0["outer_iters"],
                                           true_resid=s0["true_resid"],
                                           kernel_avg_us=[round(v, 2) for v in us],
                                           kernel_gbs=[round(v, 1) for v in gbs],
                                           whole_job_gbs=round(s0["iters"] * per_iter / t / 1e9, 1))
            log(f"{fname} {pname}: {t:.3f} s, {s0['iters']} iterations, kernels {[round(v, 1) for v in us]} us")
    d = res["dense_fp16s"]
    out = {
        "metric": METRIC, "value": d["whole_job_gbs"], "unit": "GB/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(d["seconds"] * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{dims[0]}x{dims[1]}x{dims[2]}x{dims[3]} Ls={Ls}: Cayley form vs dense form, "
                               f"H(m2)-Delta_+(m1,m2)P_+ m1={m1} m2={m2}, true residual 1e-10",
                   "lattice": list(dims), "Ls": Ls},
        "forms": res,
        "cayley_speedup_fp64": round(res["dense_fp64"]["seconds"] / res["cayley_fp64"]["seconds"], 3),
        "cayley_speedup_fp16s": round(res["dense_fp16s"]["seconds"] / res["cayley_fp16s"]["seconds"], 3),
    }
    ctx.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS) + ["batched", "learned", "force", "heatbath", "gparity", "dense", "c5"])
    ap.add_argument("--batched-iters", type=int, default=64)
    ap.add_argument("--inner", default="fp16s", choices=sorted(PREC))
    ap.add_argument("--inner-tol", type=float, default=0.0)
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP64 reference solve")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mall", action="store_true", help="skip the Dslash on a field larger than the MALL")
    ap.add_argument("--no-converge", action="store_true",
                    help="batched workload: skip the solves to 1e-10 (batched and 12 plain FP64)")
    ap.add_argument("--train-fields", type=int, default=8)
    ap.add_argument("--held-fields", type=int, default=8)
    ap.add_argument("--pairs-per-field", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-2)
    ap.add_argument("--channels", default="1,4,1", help="learned workload: channels of B, 1,...,1")
    ap.add_argument("--loss", default="residual", choices=["residual", "error"],
                    help="network loss: |A N(r) - r|^2/|r|^2 (residual) or |N(r) - e|^2/|e|^2 (error)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device-to-device copy (known bytes) to calibrate HBM counters")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the solver runs on a single GPU; --gpus must be 1 (no multi-GPU path)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1706_05843_amd import eofa, synth

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        print("bench: calibration copy done (3 x 1 GiB device-to-device)", file=sys.stderr, flush=True)

    if args.workload == "batched":
        bench_batched(args, eofa, synth, torch, np)
        return
    if args.workload == "learned":
        bench_learned(args, eofa, synth, torch, np)
        return
    if args.workload == "force":
        bench_force(args, eofa, synth, torch, np)
        return
    if args.workload == "heatbath":
        bench_heatbath(args, eofa, synth, torch, np)
        return
    if args.workload == "gparity":
        bench_gparity(args, eofa, synth, torch, np)
        return
    if args.workload == "dense":
        bench_dense(args, eofa, synth, torch, np)
        return
    if args.workload == "c5":
        bench_c5(args, eofa, synth, torch, np)
        return

    dims, Ls, eps, m1, gseed, sseed = WORKLOADS[args.workload]
    m2 = 1.0
    print(f"bench: workload {args.workload} dims={dims} Ls={Ls} eps={eps}", file=sys.stderr, flush=True)
    U = torch.from_numpy(synth.gauge_field(dims, eps, gseed)).cuda()
    phi = torch.from_numpy(synth.fermion(dims, Ls, sseed, nrhs=1)).cuda()
    psi = torch.zeros_like(phi)
    ctx = eofa.Context(eofa.make_action(dims, Ls, 1.8, 1.5, 0.5), U)
    system = [(m2, m1, m2, -1.0, +1)]  # H(m2) - Delta_+(m1, m2) P_+
    prec = PREC[args.inner]
    Vh = int(np.prod(dims)) // 2
    Nh = Vh * Ls

    def solve(p, profile=0, keep=1):
        prm = eofa.make_params(tol=1e-10, inner_prec=p, inner_tol=args.inner_tol, profile=profile,
                               keep_direction=keep)
        rc, st = ctx.eofa_cg_solve(system, phi, psi, prm)
        if rc != eofa.EOFA_OK:
            raise RuntimeError(f"solve failed rc={rc} stats={st}")
        return st[0]

    plain = None
    if not args.no_plain:
        solve(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = solve(0)
        torch.cuda.synchronize()
        plain = dict(seconds=time.perf_counter() - t0, iters=st["iters"], true_resid=st["true_resid"])
        print(f"bench: plain FP64 solve {plain}", file=sys.stderr, flush=True)

    restart = None
    if prec != 0:  # the same solve with plain defect correction (each pass restarts CG)
        solve(prec, keep=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = solve(prec, keep=0)
        torch.cuda.synchronize()
        restart = dict(time_to_solution_s=round(time.perf_counter() - t0, 5), iters=st["iters"],
                       outer_iters=st["outer_iters"], true_resid=st["true_resid"])
        print(f"bench: restarted defect correction {restart}", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        solve(prec, profile=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [solve(prec, profile=1) for _ in range(args.steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt * 1e3 / args.steps
    print(f"bench: {args.steps} steps {ms:.2f} ms/step", file=sys.stderr, flush=True)

    # whole-job Dslash throughput: the hop's compulsory bytes of every inner hop
    # launch (4 per iteration, 2 more per outer pass for M^dag r) / wall time;
    # the same with each launch's fused bytes is reported beside it
    iters = sum(s["iters"] for s in stats)
    outer = sum(s["outer_iters"] for s in stats)
    total_bytes = (4 * iters + 2 * outer) * hop_bytes(prec, Ls, Nh)
    value = total_bytes / dt / 1e9
    fused_total = (iters * sum(role_bytes(k, prec, Ls, Nh) for k in range(4))
                   + outer * (role_bytes(2, prec, Ls, Nh) + role_bytes(3, prec, Ls, Nh)))

    # dominant kernel: the hop role with the largest timed share; its achieved
    # bandwidth counts the hop's own compulsory bytes (input and output spinor,
    # links), the fused bytes of its epilogue reported beside it
    hop_ms = np.sum([s["hop_ms"] for s in stats], axis=0)
    timed = sum(s["hop_timed"] for s in stats)
    avg_us = [h / max(timed, 1) * 1e3 for h in hop_ms]
    dom = int(np.argmax(hop_ms))
    avg_ms = avg_us[dom] * 1e-3
    dom_bytes = hop_bytes(prec, Ls, Nh)
    achieved = dom_bytes / (avg_ms * 1e-3) / 1e9
    traffic = traffic_from_profile(args.workload, args.inner, dom)
    # Wilson-hop flops: 1320 per 4D site per Ls slice (the conventional count, per hop launch)
    flop_per_launch = 1320.0 * Nh
    gflops_dom = flop_per_launch / (avg_ms * 1e-3) / 1e9
    gflops_job = 4 * iters * flop_per_launch / dt / 1e9
    roles = []
    for k in range(4):
        t = avg_us[k] * 1e-6
        hb, fb = hop_bytes(prec, Ls, Nh) / t / 1e9, role_bytes(k, prec, Ls, Nh) / t / 1e9
        roles.append(dict(kernel=ROLE_NAMES[k], avg_launch_us=round(avg_us[k], 2), hop_GBs=round(hb, 1),
                          hop_frac=round(hb / HBM_PEAK_GBS, 4), fused_GBs=round(fb, 1),
                          fused_frac=round(fb / HBM_PEAK_GBS, 4)))
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                kernel=ROLE_NAMES[dom], avg_launch_us=round(avg_us[dom], 2),
                algorithmic_bytes_per_launch=int(dom_bytes),
                bytes_model="hop compulsory bytes: input and output spinor once, links once per launch",
                fused_bytes_per_launch=int(role_bytes(dom, prec, Ls, Nh)),
                fused_frac=round(role_bytes(dom, prec, Ls, Nh) / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                all_roles=roles)
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if prec else "f64", "data": "synthetic",
        "precision": {"fp16s": "inner CG: FP16 storage + per-site FP32 scale, FP32 arithmetic; FP64 outer "
                               "defect correction with reliable updates (search direction kept across passes)",
                      "fp32": "inner CG FP32; FP64 outer defect correction with reliable updates",
                      "fp64": "FP64 throughout"}[args.inner],
        "config": {"workload": f"{dims[0]}x{dims[1]}x{dims[2]}x{dims[3]} Ls={Ls} Mobius b5=1.5 c5=0.5 M5=1.8, "
                               f"links exp(i {eps} H), system H(m2)-Delta_+(m1,m2)P_+ m1={m1} m2={m2}, "
                               f"1 Gaussian RHS, true residual 1e-10",
                   "lattice": list(dims), "Ls": Ls, "nrhs": 1, "inner": args.inner},
        "dslash_gflops": {"dominant_kernel": round(gflops_dom, 1), "whole_job": round(gflops_job, 1),
                          "flop_model": "1320 flop per 4D site per Ls slice per hop launch (4 launches per iteration)"},
        "value_fused_bytes_GBs": round(fused_total / dt / 1e9, 1),
        "time_to_solution_s": round(ms / 1e3, 5),
        "iters": stats[-1]["iters"], "outer_iters": stats[-1]["outer_iters"],
        "true_resid": stats[-1]["true_resid"],
        "launch_shape": {"waves": stats[-1]["waves"], "rhs_block": stats[-1]["rhs_block"]},
        "roofline": roof,
    }
    if restart is not None:
        out["restarted_defect_correction"] = restart
    if plain is not None:
        out["plain_fp64"] = dict(time_to_solution_s=round(plain["seconds"], 5), iters=plain["iters"],
                                 true_resid=plain["true_resid"])
        out["speedup_vs_plain_fp64"] = round(plain["seconds"] / (ms / 1e3), 3)
    ctx.close()
    del phi, psi, U
    torch.cuda.empty_cache()
    if not args.no_mall:
        print("bench: Dslash on a field larger than the MALL (24^3x64, Ls=12)", file=sys.stderr, flush=True)
        out["dslash_beyond_mall"] = dslash_beyond_mall(eofa, synth, torch, np)
        torch.cuda.empty_cache()
    if not args.no_cpu:
        print("bench: the same solve on 4^4 x Ls=8 on the GPU and with the CPU oracle", file=sys.stderr, flush=True)
        out["gpu_c1_time_to_solution"] = gpu_c1(eofa, synth, torch)
        out["cpu_baseline"] = cpu_baseline(dims, Ls, eps, m1, gseed, sseed,
                                           plain_iters=plain["iters"] if plain is not None else None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
