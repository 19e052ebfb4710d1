"""Benchmark of the Wilson-clover / C* / SAP-GCR hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-solve] [--no-cpu]

Prints one JSON line.  `value` is the achieved bandwidth of the Dirac
operator D = hop + Pauli in FP64 on the 64 x 32^3 lattice with C* boundaries
in x, y, z (4,194,304 extended sites): algorithmic bytes of one application
(each field read once: in and out spinors, the hopping links W = U z^qhat --
only the physical half's when the kernel reads the C* mirror links at their
physical partners -- and the Pauli term) divided by the average time of one
application, measured with
HIP events over K back-to-back applications on the launch stream.  A "step"
is one such application; inputs are resident in HBM.  The other precisions,
the mixed-precision versus FP64 solve rates and the oracle timed on the host
cores are reported alongside.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Dw GB/s (% HBM peak); mixed-prec batched solves/sec & p99 vs FP64 @1e-10"
HBM_PEAK_GBS = 8000.0

# algorithmic bytes per extended site of one D application with the phase
# folded into the links: spinor in + out (24 reals each), W links (4 x 18
# reals), Pauli term (2 x 36 reals); FP16S adds one fp32 scale per spinor site.
BYTES_PER_SITE = {0: 48 * 8 + 72 * 8 + 72 * 8, 1: 48 * 4 + 72 * 4 + 72 * 4,
                  2: 48 * 2 + 8 + 72 * 2 + 72 * 2, 3: 48 * 2 + 72 * 2 + 72 * 2}
# link bytes per extended site (4 x 18 reals): with the mirror-fused link
# reads on a C* lattice (variant bit 64) the mirror half's links are read at
# their physical partners, so one application needs half of them
LINK_BYTES = {0: 72 * 8, 1: 72 * 4, 2: 72 * 2, 3: 72 * 2}
FLOPS_PER_SITE = 1320 + 552 + 48   # hops + two 6x6 Hermitian blocks + combine


def site_bytes(prec, choice):
    """Algorithmic bytes per extended site for the kernel variant `choice`."""
    mirror = (choice & 16) and (choice & 64)
    return BYTES_PER_SITE[prec] - (LINK_BYTES[prec] // 2 if mirror else 0)


# HBM bytes per FP64 launch from the calibrated FETCH_SIZE + WRITE_SIZE
# counters (profiles/dirac_64x32c_hbm_counters.md), valid only for the kernel
# sources they were taken on (hash of the files below) and for the variant
# the autotuner picked there (hop group + 16 LDS + 32 non-temporal + 64 mirror).
KERNEL_FILES = ["dirac.hip", "dirac_site.h", "qxd_impl.h"]
TRAFFIC = {("34a0479e4cb9cdce", 113): 8.126e9, ("34a0479e4cb9cdce", 114): 8.125e9,
           ("34a0479e4cb9cdce", 241): 8.128e9, ("34a0479e4cb9cdce", 242): 8.119e9}


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_FILES:
        with open(os.path.join(ROOT, "paper_1710_08839_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]
PREC_NAME = {0: "f64", 1: "f32", 2: "f16s", 3: "bf16"}


def kernel_name(choice, prec):
    """The Dirac kernel the autotuner picked (hop group, LDS staging,
    non-temporal streams), as its template appears in profiler traces."""
    if choice == 0:
        return "dirac_kernel (not tuned)"
    g, lds, nt = choice & 15, bool(choice & 16), bool(choice & 32)
    if lds:
        name = "dirac_wave_kernel" if choice & 128 else "dirac_lds_kernel"
        return (f"{name}<{prec}, 0, {g}, {'true' if nt else 'false'}>"
                + (" (mirror-fused links)" if choice & 64 else ""))
    return f"dirac_kernel<{prec}, 0, {g}>"
_T0 = time.perf_counter()


def log(msg):
    print(f"[bench {time.perf_counter() - _T0:7.1f}s] {msg}", file=sys.stderr, flush=True)


def time_applies(field, q, prec, nrhs_bufs, steps, warmup):
    import torch
    from paper_1710_08839_amd import qxd
    nb = field.spinor_bytes(prec)
    bufs = [torch.empty(nb // 4, dtype=torch.float32, device="cuda") for _ in range(2 * nrhs_bufs)]
    src = torch.empty(field.volume * 24, dtype=torch.float64, device="cuda").normal_()
    for k in range(nrhs_bufs):
        field.pack(prec, src, bufs[2 * k])
    stream = torch.cuda.current_stream()
    for i in range(warmup):
        k = i % nrhs_bufs
        field.apply(q, qxd.OP_D, prec, bufs[2 * k], bufs[2 * k + 1], native=True, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(steps):
        k = i % nrhs_bufs
        field.apply(q, qxd.OP_D, prec, bufs[2 * k], bufs[2 * k + 1], native=True, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    return ms


CPU_DIMS = (16, 8, 8, 8)       # the bounded sample of the 64x32^3 C* workload for the oracle's D
CFG2 = dict(dims=(64, 32, 32, 32), seed=20171002, eps=0.25, sigma=0.15, kappa=0.1365, q=-1 / 3, csw=1.9,
            src_seed=1003)
SAMPLE_SEED = 5


def cfg2_sample_sites(V):
    """Sampled extended sites of the 64x32^3 C* lattice at which the GPU's D
    is compared with the oracle (and the first and last site)."""
    rng = np.random.default_rng(SAMPLE_SEED)
    return np.concatenate([rng.choice(V, 64, replace=False), [0, V - 1]])


def _cpu_share():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_d_worker(args):
    """One process: apply the oracle's D to its own source for budget_s
    seconds (single-threaded numpy); returns (applications, seconds)."""
    seed, budget_s = args
    from threadpoolctl import threadpool_limits

    from oracle import Lattice
    from oracle import dirac as od
    from oracle import fields as of
    from paper_1710_08839_amd import synth
    with threadpool_limits(limits=1):
        lat = Lattice(CPU_DIMS, cstar=3)
        u, a = synth.gauge_field(CPU_DIMS, 20171002, 0.25, 0.15)
        ue, ae = of.extend_gauge(lat, u, a)
        op = od.build_operator(lat, ue, ae, 0.1365, q=-1 / 3, csw=1.9)
        x = synth.source(CPU_DIMS, 3, seed)
        op.apply(x)
        n, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            op.apply(x)
            n += 1
        return n, time.perf_counter() - t0, lat.V


def cpu_baseline_child(out_npy, budget_s=8.0):
    """The CPU leg, run in a child process that never touches the GPU: the
    oracle's D timed on one core and on every core of the CPU share, the
    per-site D at the 64x32^3 C* shape (clover term evaluated on the fly, as
    the oracle's per-site form does), the even-odd GCR solve of the 8x8^3
    periodic SU(3) workload, and the oracle's D at the sampled 64x32^3 sites
    (saved to out_npy for the GPU error report)."""
    import multiprocessing as mp

    from threadpoolctl import threadpool_limits

    from oracle import Lattice
    from oracle import dirac as od
    from oracle import fields as of
    from oracle import solvers as osv
    from paper_1710_08839_amd import synth
    res = {"cpu_model": _cpu_model()}
    ncores = _cpu_share()
    ctx = mp.get_context("fork")
    with ctx.Pool(1) as pool:
        n1, t1, V = pool.map(_oracle_d_worker, [(1003, budget_s)])[0]
    with ctx.Pool(ncores) as pool:
        outs = pool.map(_oracle_d_worker, [(1003 + k, budget_s) for k in range(ncores)])
    napp = sum(o[0] for o in outs)
    wall = max(o[1] for o in outs)
    gb1 = BYTES_PER_SITE[0] * V * n1 / t1 / 1e9
    gbn = BYTES_PER_SITE[0] * V * napp / wall / 1e9
    res["one_core"] = {"value": round(gb1, 4), "unit": "GB/s", "cores": 1,
                       "msites_per_s": round(V * n1 / t1 / 1e6, 4), "applications": n1, "seconds": round(t1, 2)}
    res["all_cores"] = {"value": round(gbn, 4), "unit": "GB/s", "cores": ncores,
                        "msites_per_s": round(V * napp / wall / 1e6, 4), "applications": napp,
                        "seconds": round(wall, 2)}
    with threadpool_limits(limits=1):
        # the 64x32^3 C* lattice: oracle D at sampled sites (error report and
        # per-site cost with the clover term built on the fly)
        c = CFG2
        lat = Lattice(c["dims"], cstar=3)
        u, a = synth.gauge_field(c["dims"], c["seed"], c["eps"], c["sigma"])
        ue, ae = of.extend_gauge(lat, u, a)
        del u, a
        x = synth.source(c["dims"], 3, c["src_seed"])
        sites = cfg2_sample_sites(lat.V)
        kw = dict(q=c["q"], csw=c["csw"], csw_u1=1.0)
        expect = od.apply_at_sites(lat, ue, ae, x, sites, c["kappa"], **kw)
        np.save(out_npy, expect)
        rng = np.random.default_rng(7)
        probe = rng.choice(lat.V, 4096, replace=False)
        t0 = time.perf_counter()
        od.apply_at_sites(lat, ue, ae, x, probe, c["kappa"], **kw)
        dt = time.perf_counter() - t0
        res["cfg2_per_site"] = {"us_per_site": round(dt / len(probe) * 1e6, 2), "sites": len(probe), "cores": 1,
                                "what": "oracle per-site D at 64x32^3 C* (hops + clover term built per site)"}
        del ue, ae, x, lat
        # the 8x8^3 periodic SU(3) even-odd GCR solve to 1e-10
        d0 = (8, 8, 8, 8)
        lat0 = Lattice(d0, cstar=0)
        u0, _ = synth.gauge_field(d0, 20171000, 0.3)
        ue0, _ = of.extend_gauge(lat0, u0, None)
        op0 = od.build_operator(lat0, ue0, None, 0.124, csw=1.0)
        eta0 = synth.source(d0, 0, 1000)
        t0 = time.perf_counter()
        psi0, it0 = osv.solve_eo(op0, eta0, 1e-10, nkv=16)
        dt0 = time.perf_counter() - t0
        r0 = od.norm(eta0 - op0.apply(psi0)) / od.norm(eta0)
        res["eo_gcr_8x8c3"] = {"seconds": round(dt0, 3), "gcr_iterations": int(it0), "true_resid": float(r0),
                               "cores": 1}
    return res


def cpu_baseline_run():
    """Run the CPU leg in a child process (forked workers need a parent that
    has not touched the GPU); returns (cpu_baseline record, oracle values at
    the sampled 64x32^3 sites or None)."""
    import subprocess
    import tempfile
    fd, path = tempfile.mkstemp(suffix=".npy")
    os.close(fd)
    try:
        p = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-child", path],
                           capture_output=True, text=True, timeout=900)
        if p.returncode != 0:
            log(f"cpu baseline child failed: {p.stderr[-2000:]}")
            return None, None
        res = json.loads(p.stdout.strip().splitlines()[-1])
        expect = np.load(path)
    finally:
        os.unlink(path)
    one, alln = res["one_core"], res["all_cores"]
    rec = {"value": alln["value"], "unit": "GB/s", "cores": alln["cores"], "kind": "oracle",
           "sample": f"FP64 numpy oracle D (stored clover term) on 16x8^3 C* (16384 extended sites), one "
                     f"source per process in {alln['cores']} single-threaded processes for "
                     f"{alln['seconds']} s: {alln['applications']} applications, {alln['msites_per_s']} Msite/s; "
                     f"algorithmic bytes as for the GPU FP64 D without mirror fusion (1536 B/site)",
           "cpu_model": res["cpu_model"], "one_core": one,
           "cfg2_per_site": res["cfg2_per_site"], "eo_gcr_8x8c3": res["eo_gcr_8x8c3"]}
    return rec, expect


def solve_rates(ctx, nsrc, nsrc_fp64, dims=(48, 24, 24, 24)):
    """48 x 24^3 with C*: nsrc spin-colour point sources at the origin x 2
    charges x 2 kappas, solved to a true FP64 residual of 1e-10 by the batched
    mixed-precision SAP-GCR (all right-hand sides in one call) and, one after
    another, by the plain FP64 even-odd GCR (a sample of nsrc_fp64 sources per
    operator: its rate is per right-hand side)."""
    import torch
    from paper_1710_08839_amd import qxd, synth
    u, a = synth.gauge_field(dims, 20171003, 0.25, 0.15)
    f = qxd.Field(ctx, dims, u, a, cstar=3)
    del u, a
    ops = [qxd.quark(k, q, 1.9, 1.0) for q in (2 / 3, -1 / 3) for k in (0.1360, 0.1365)]
    V = f.volume

    def sources(n):
        return [synth.point_source(V, 0, s // 3 % 4, s % 3) for s in range(n)]

    out = {}
    # Krylov lengths: the measured best for each inner precision on this
    # batch (FP32 slots are twice the size of FP16 ones, so 48 of them do not
    # all fit in HBM at once and the longer cycle pays off)
    legs = [("mixed_sap_gcr_f32", qxd.solver(kind=qxd.SAP_GCR, tol=1e-10, nkv=32, ncy=4, nmr=4,
                                              inner_prec=qxd.F32), nsrc),
            ("mixed_sap_gcr_f16s", qxd.solver(kind=qxd.SAP_GCR, tol=1e-10, nkv=24, ncy=4, nmr=4,
                                               inner_prec=qxd.F16S), nsrc),
            ("fp64_eo_gcr", qxd.solver(kind=qxd.EO_GCR, tol=1e-10, nkv=64, maxiter=20000), nsrc_fp64)]
    for name, s, ns in legs:
        if ns <= 0:
            continue
        eta = torch.from_numpy(np.stack(sources(ns) * len(ops))).cuda()
        nrhs = eta.shape[0]
        psi = torch.empty_like(eta)
        # warm-up on a small right-hand side set: builds operators and tunes kernels
        f.solve(ops[0], qxd.solver(kind=s.kind, tol=1e-4, nkv=s.nkv, ncy=s.ncy, nmr=s.nmr,
                                   inner_prec=s.inner_prec), eta[:1], psi[:1], check=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, info = f.solve(ops, s, eta, psi, nrhs=nrhs, check=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        log(f"solve {name}: {nrhs} rhs in {dt:.2f} s, status {st}")
        out[name] = {"solves_per_s": round(nrhs / dt, 4), "seconds": round(dt, 3), "nrhs": nrhs,
                     "nkv_ncy_nmr": [s.nkv, s.ncy, s.nmr],
                     "status": st, "max_true_resid": max(i.true_resid for i in info),
                     "inner_iters_per_operator": [i.inner_iters for i in info][::ns],
                     "outer_iters_per_operator": [i.outer_iters for i in info][::ns]}
        del eta, psi
    f.release()
    base = out.get("fp64_eo_gcr", {}).get("solves_per_s")
    for k in out:
        if base:
            out[k]["speedup_vs_fp64_eo_gcr"] = round(out[k]["solves_per_s"] / base, 2)
    out["workload"] = (f"{dims[0]}x{dims[1]}^3 C* (1327104 extended sites), point sources x (q, kappa) in "
                       f"{{2/3,-1/3}} x {{0.1360,0.1365}}, csw=1.9; batched SAP-GCR: {nsrc} sources x 4 "
                       f"operators in one call; FP64 even-odd GCR(64): {nsrc_fp64} source(s) x 4 "
                       f"operators one after another")
    return out


def single_solve(f, q, s, eta):
    """One right-hand side to a true FP64 residual of 1e-10; the residual is
    the library's own FP64 ||eta - D psi|| / ||eta|| (the FP64 operator is
    tested against the oracle to 1e-12)."""
    import torch
    from paper_1710_08839_amd import qxd
    psi = torch.empty_like(eta)
    # warm-up: builds the operator in the inner precision and tunes its kernels
    f.solve(q, qxd.solver(kind=s.kind, tol=1e-3, nkv=s.nkv, ncy=s.ncy, nmr=s.nmr, inner_prec=s.inner_prec),
            eta, psi, check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, info = f.solve(q, s, eta, psi, check=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    i = info[0]
    return {"seconds": round(dt, 3), "status": st, "outer_iters": i.outer_iters, "inner_iters": i.inner_iters,
            "true_resid": i.true_resid}


def single_rhs_32x16(ctx):
    """32 x 16^3 with C* in x, y, z (eps 0.3, A ~ N(0, 0.15), kappa 0.124,
    csw 1.0), periodic and open time, one Gaussian source per charge:
    SAP-GCR with 4^4 blocks and an FP32 or an FP64 inner solver."""
    import torch
    from paper_1710_08839_amd import qxd, synth
    dims = (32, 16, 16, 16)
    u, a = synth.gauge_field(dims, 20171001, 0.3, 0.15)
    out = {}
    for tbc, tname in ((0, "periodic"), (1, "open")):
        f = qxd.Field(ctx, dims, u, a, cstar=3, time_bc=tbc)
        for q, seed in ((2 / 3, 1001), (-1 / 3, 1002)):
            eta = torch.from_numpy(synth.source(dims, 3, seed)).cuda()
            for name, prec in (("f32_inner", qxd.F32), ("f64_inner", qxd.F64)):
                s = qxd.solver(kind=qxd.SAP_GCR, tol=1e-10, nkv=24, ncy=4, nmr=4, inner_prec=prec)
                r = single_solve(f, qxd.quark(0.124, q, 1.0, 1.0), s, eta)
                out[f"{tname} q={q:+.3f} {name}"] = r
                log(f"32x16^3 {tname} q={q:+.3f} {name}: {r['seconds']} s, outer {r['outer_iters']}, "
                    f"inner {r['inner_iters']}, resid {r['true_resid']:.2e}")
        f.release()
    return out


def single_rhs_8x8(ctx):
    """8 x 8^3 periodic SU(3) (eps 0.3, kappa 0.124, csw 1.0), one Gaussian
    source: the plain FP64 even-odd GCR to 1e-10, the workload the oracle's
    solve is timed on."""
    import torch
    from paper_1710_08839_amd import qxd, synth
    dims = (8, 8, 8, 8)
    u, _ = synth.gauge_field(dims, 20171000, 0.3)
    f = qxd.Field(ctx, dims, u, None, cstar=0)
    eta = torch.from_numpy(synth.source(dims, 0, 1000)).cuda()
    r = single_solve(f, qxd.quark(0.124, 0.0, 1.0, 1.0), qxd.solver(kind=qxd.EO_GCR, tol=1e-10, nkv=16), eta)
    f.release()
    log(f"8x8^3 EO-GCR: {r['seconds']} s, {r['inner_iters']} iterations, resid {r['true_resid']:.2e}")
    return {"fp64_eo_gcr": r}


# Algorithmic flops of one SAP colour pass on one 4^4 block (256 sites, 128
# of each parity) and one right-hand side, counted from the block algorithm
# with the per-hop and per-Pauli costs of the D count: a hop (projection,
# SU(3) product on the two-spin half spinor, reconstruction and
# accumulation) 165 = 1320 / 8, a Pauli block application (two 6x6 Hermitian
# blocks) 552; complex 12-component axpy 96, dot 96, norm 48, add 24.  An
# interior site of a 4^4 block has 6 of its 8 neighbours in the block.
HOP, PAULI = 165, 552


def sap_block_flops(nmr):
    face = 512 * HOP                                        # 8 faces x 64 sites, one hop each
    prep = 128 * (PAULI + 6 * HOP + 24)                     # rho_e = r_e - D_eo D_oo^-1 r_o
    mr = nmr * 128 * (12 * HOP + 2 * PAULI + 24 + 96 + 48 + 96 + 96)  # D^ s, dots, two axpys
    recon = 128 * (6 * HOP + 24 + PAULI)                    # v_o = D_oo^-1 (r_o - D_oe v_e)
    resid = 256 * (6 * HOP + PAULI + 24) + 256 * 24         # r -= D_Lambda v, psi += v
    return face + prep + mr + recon + resid


FP32_VALU_PEAK_TFLOPS = 78.6  # 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz, no packed FP32


def sap_leg(f, q, nmr=4, reps=20):
    """One colour pass of the paired SAP block solver (two right-hand sides
    sharing the operator per work-group, the kernel that dominates the batched
    solve) on the 64 x 32^3 lattice, timed with HIP events over reps launches,
    against the FP32 VALU peak."""
    from paper_1710_08839_amd import qxd
    nblocks = f.volume // 256
    flops = sap_block_flops(nmr) * (nblocks // 2) * 2
    out = {}
    for name, prec in (("f32", qxd.F32), ("f16s", qxd.F16S)):
        ms = f.sap_pair_pass_ms(q, prec, nmr=nmr, npair=1, reps=reps)
        tf = flops / (ms * 1e-3) / 1e12
        out[name] = {"kernel": f"sapq_pair_kernel<{prec}>", "ms_per_pass": round(ms, 4),
                     "TFLOP/s": round(tf, 2), "frac": round(tf / FP32_VALU_PEAK_TFLOPS, 4)}
        log(f"SAP pair pass {name}: {ms:.4f} ms, {tf:.1f} TFLOP/s")
    out.update({"bound": "alu", "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "flops_per_pass": flops, "flops_per_block_rhs": sap_block_flops(nmr), "nmr": nmr,
                "workload": "64x32^3 C*, q=-1/3, kappa=0.1365, csw=1.9; colour 0 (8192 blocks of 4^4), 2 right-hand "
                            "sides, face update included, synthetic vectors"})
    return out


# zeros and poles of the rational approximation of the QCD2 / QCD3 runs
# (Table 2 of the paper), for the multi-shift leg
TABLE2_MU = [1.2383e+01, 4.8370e+00, 2.3515e+00, 1.1994e+00, 6.1927e-01, 3.2079e-01, 1.6632e-01, 8.6246e-02,
             4.4718e-02, 2.3170e-02, 1.1973e-02, 6.1273e-03, 3.0301e-03, 1.3855e-03]


def multishift_leg(f, iters=(20, 60)):
    """Multi-shift CG on D^dag D^ of the 64 x 32^3 field with the 14 poles
    mu_j^2 of Table 2 as shifts: two runs capped at iters[0] and iters[1]
    iterations (no shift converges that early on this operator), timed with
    wall clock around the synchronising calls; the difference over the extra
    iterations is the cost of one iteration with all 14 shifts active."""
    import torch
    from paper_1710_08839_amd import qxd, synth
    dims = f.lat.dims[:]
    q = qxd.quark(CFG2["kappa"], CFG2["q"], CFG2["csw"], 1.0)
    eta = torch.from_numpy(synth.source(tuple(dims), 3, CFG2["src_seed"])).cuda()
    shifts = np.array(TABLE2_MU) ** 2
    psi = torch.empty((len(shifts),) + tuple(eta.shape), dtype=eta.dtype, device="cuda")
    f.multishift(q, shifts, eta, psi, tol=1e-10, maxiter=3, check=False)  # builds and tunes
    t = []
    for k in iters:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, info = f.multishift(q, shifts, eta, psi, tol=1e-10, maxiter=k, check=False)
        t.append(time.perf_counter() - t0)
    ms_it = (t[1] - t[0]) / (iters[1] - iters[0]) * 1e3
    V = f.volume
    # per iteration: the shifted update reads r, p, x_j, p_j and writes p,
    # x_j, p_j (FP64 even-site spinors of 192 B per site)
    upd = (3 + 4 * len(shifts)) * (V // 2) * 192
    del psi, eta
    log(f"multi-shift CG, 14 shifts: {ms_it:.2f} ms per iteration")
    return {"shifts": len(shifts), "ms_per_iteration": round(ms_it, 3),
            "update_bytes_per_iteration": upd,
            "workload": "64x32^3 C*, q=-1/3, kappa=0.1365, csw=1.9, shifts mu_j^2 of Table 2 (14), FP64"}


def single_rhs_64x32(f):
    """The 64 x 32^3 field of the D leg (q = -1/3, kappa 0.1365, csw 1.9), one
    Gaussian source: SAP-GCR with FP16+scale or BF16 inner storage (FP32
    arithmetic) and FP64 outer defect correction."""
    import torch
    from paper_1710_08839_amd import qxd, synth
    dims = (64, 32, 32, 32)
    eta = torch.from_numpy(synth.source(dims, 3, 1003)).cuda()
    q = qxd.quark(0.1365, -1 / 3, 1.9, 1.0)
    out = {}
    for name, prec in (("f16s_inner", qxd.F16S), ("bf16_inner", qxd.BF16)):
        s = qxd.solver(kind=qxd.SAP_GCR, tol=1e-10, nkv=24, ncy=4, nmr=4, inner_prec=prec)
        r = single_solve(f, q, s, eta)
        out[name] = r
        log(f"64x32^3 {name}: {r['seconds']} s, outer {r['outer_iters']}, inner {r['inner_iters']}, "
            f"resid {r['true_resid']:.2e}")
    return out


def dfl_leg(f, ns=16, ninv=30, nkv=32):
    """Locally deflated SAP-GCR on the 64 x 32^3 field of the D leg (q = -1/3,
    kappa 0.1365, csw 1.9), one Gaussian source: the deflation subspace's
    setup time, then the deflated solve and the plain SAP-GCR on the same
    source, both with FP32 inner storage, FP64 defect correction and the same
    Schwarz parameters (4^4 blocks, ncy 4, nmr 4, nkv 32)."""
    import torch
    from paper_1710_08839_amd import qxd, synth
    dims = (64, 32, 32, 32)
    eta = torch.from_numpy(synth.source(dims, 3, 1003)).cuda()
    q = qxd.quark(0.1365, -1 / 3, 1.9, 1.0)
    sap = single_solve(f, q, qxd.solver(kind=qxd.SAP_GCR, tol=1e-10, nkv=nkv, ncy=4, nmr=4, inner_prec=qxd.F32), eta)
    log(f"64x32^3 SAP-GCR (fp32 inner): {sap}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f.dfl_setup(q, ns=ns, ninv=ninv, ncy=4, nmr=4, seed=2017)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    dfl = single_solve(f, q, qxd.solver(kind=qxd.DFL_SAP_GCR, tol=1e-10, nkv=nkv, ncy=4, nmr=4,
                                        inner_prec=qxd.F32), eta)
    st = f.dfl_stats(q)  # the warm-up and the timed solve
    log(f"64x32^3 deflated SAP-GCR: setup {setup_s:.2f} s, {dfl}")
    return {"setup_s": round(setup_s, 3), "deflated": dfl, "sap_gcr": sap,
            "subspace": {"ns": ns, "ninv": ninv, "ncy": 4, "nmr": 4, "little_tol": 0.2, "little_nkv": 48},
            "little": {"applications": st[0], "iterations": st[1], "max_per_solve": st[2]},
            "workload": "64x32^3 C*, q=-1/3, kappa=0.1365, csw=1.9, Gaussian source (seed 1003), tol 1e-10"}


def stream_gbs(reads_per_write, dst_bytes=49152 * 21845, reps=10):
    """The library's streaming probe (reads_per_write bytes read per byte
    written, each once), timed with HIP events: the practical HBM ceiling for
    that read/write mix next to the kernels' rates."""
    import torch
    from paper_1710_08839_amd import qxd
    a = torch.empty(reads_per_write * dst_bytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty(dst_bytes // 4, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    qxd.stream_probe(a, b, dst_bytes, reads_per_write, stream=stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        qxd.stream_probe(a, b, dst_bytes, reads_per_write, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return round((reads_per_write + 1) * dst_bytes / (ms * 1e-3) / 1e9, 1)


SERVE_SIZES = [(8, 8, 8, 8), (32, 16, 16, 16), (48, 24, 24, 24), (64, 32, 32, 32)]


def serve_fields(ctx, inner_prec, nkv):
    """The resident fields of the four serving lattice sizes (C*), with one
    loose solve per size first so that the kernels of each volume are tuned
    before any stream is timed (operators are not built ahead: the stream's
    requests build their own)."""
    import torch
    from paper_1710_08839_amd import qxd, synth
    fields = []
    for i, d in enumerate(SERVE_SIZES):
        u, a = synth.gauge_field(d, 20171010 + i, 0.25, 0.15)
        fields.append(qxd.Field(ctx, d, u, a, cstar=3))
        del u, a
    for f in fields:
        e = torch.from_numpy(synth.source(tuple(f.lat.dims[:]), 3, 7)[None]).cuda()
        f.solve(qxd.quark(0.13, 2 / 3, 1.9, 1.0), qxd.solver(kind=qxd.SAP_GCR, tol=1e-3, nkv=nkv,
                                                             inner_prec=inner_prec), e, torch.empty_like(e),
                check=False)
    torch.cuda.synchronize()
    return fields


def serve_stream(ctx, nreq, max_rhs, rate, inner_prec, seed=4242, nkv=32):
    """A short serving stream: nreq Poisson requests at `rate`/s over the four
    lattice sizes (C*), random charge, kappa ~ U[0.130, 0.1365], Gaussian or
    point sources, 1..max_rhs right-hand sides; returns latency statistics."""
    from paper_1710_08839_amd import qxd
    fields = serve_fields(ctx, inner_prec, nkv)
    s = qxd.solver(kind=qxd.SAP_GCR, tol=1e-10, nkv=nkv, ncy=4, nmr=4, inner_prec=inner_prec)
    reqs = draw_requests(np.random.default_rng(seed), nreq, max_rhs, rate)
    res, wall = run_stream(ctx, fields, reqs, s, limit_s=600)
    for f in fields:
        f.release()
    out = stream_stats(reqs, res, wall)
    out["stream"] = (f"{nreq} Poisson requests at {rate}/s over lattices "
                     f"{[f'{d[0]}x{d[1]}^3' for d in SERVE_SIZES]} (C*), 1-{max_rhs} RHS each, "
                     f"q in {{2/3,-1/3}}, kappa~U[0.130,0.1365], csw=1.9, Gaussian or point sources")
    return out


def draw_requests(rng, nreq, max_rhs, rate, t_start=0.0):
    """Requests of the serving workload: Poisson arrivals at `rate` (all at
    t_start if rate is None), lattice size ~U{4 sizes}, q ~U{2/3, -1/3},
    kappa ~U[0.130, 0.1365], Gaussian or point sources (p = 1/2), 1..max_rhs
    right-hand sides, source seed 5000 + j."""
    reqs, t = [], t_start
    for j in range(nreq):
        if rate:
            t += rng.exponential(1.0 / rate)
        reqs.append((t, int(rng.integers(len(SERVE_SIZES))), float(rng.choice([2 / 3, -1 / 3])),
                     float(rng.uniform(0.130, 0.1365)), int(rng.integers(1, max_rhs + 1)), bool(rng.integers(2)),
                     5000 + j))
    return reqs


def device_source(V, nrhs, point, seed):
    """nrhs synthetic sources made on the device (a request's payload): spin-
    colour point sources at a random site, or N(0, 1) real and imaginary
    parts, from a torch generator seeded with `seed`."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    if point:
        e = torch.zeros((nrhs, V * 12), dtype=torch.complex128, device="cuda")
        idx = torch.randint(0, V * 12, (nrhs,), generator=g, device="cuda")
        e[torch.arange(nrhs, device="cuda"), idx] = 1.0
        return e.view(nrhs, V, 4, 3)
    return torch.view_as_complex(torch.randn((nrhs, V, 4, 3, 2), dtype=torch.float64, generator=g,
                                             device="cuda"))


def run_stream(ctx, fields, reqs, s, budget_frac=0.6, limit_s=1e9):
    """Submit the requests at their arrival times to the serve loop and poll
    them.  A request's source and solution buffers are made on the device
    when it is submitted and freed when it completes; a request whose
    buffers do not fit waits at the client until completions free memory
    (that wait counts in its latency).  The serve budget is budget_frac of
    the device memory free at the start, leaving the rest to the buffers.
    Returns {index: (result, client wait in s)} and the wall time."""
    import torch
    from paper_1710_08839_amd import qxd
    torch.cuda.synchronize()
    free, _ = torch.cuda.mem_get_info()
    ctx.serve_start(budget_bytes=int(budget_frac * free))
    tickets, results, bufs, errors = {}, {}, {}, []
    t0 = time.perf_counter()
    j, t_log = 0, 0.0
    try:
        while len(results) < len(reqs):
            now = time.perf_counter() - t0
            if now - t_log >= 20.0:
                log(f"  stream: {j} submitted, {len(results)} of {len(reqs)} completed after {now:.0f} s")
                t_log = now
            while j < len(reqs) and reqs[j][0] <= now:
                (t_arr, fi, q, k, nrhs, point, sd) = reqs[j]
                try:
                    e = device_source(fields[fi].volume, nrhs, point, sd)
                    p = torch.empty_like(e)
                except torch.OutOfMemoryError:
                    break  # back-pressure: wait for completions
                torch.cuda.synchronize()
                tk = ctx.serve_submit(fields[fi], qxd.quark(k, q, 1.9, 1.0), s, e, p, nrhs)
                tickets[tk] = (j, time.perf_counter() - t0 - t_arr)
                bufs[tk] = (e, p)
                j += 1
            freed = False
            for tk in list(tickets):
                r = ctx.serve_poll(tk)
                if r is not None:
                    i, wait = tickets.pop(tk)
                    results[i] = (r, wait)
                    if r.status != 0:
                        errors.append(qxd.last_error()[:200])
                    del bufs[tk]
                    freed = True
            if freed:
                # hand the freed buffers back to the device (torch would keep
                # them cached, out of the library's free memory)
                torch.cuda.empty_cache()
            if time.perf_counter() - t0 > limit_s:
                break
            time.sleep(0.002)
    finally:
        ctx.serve_stop()
    wall = time.perf_counter() - t0
    for m in sorted(set(errors)):
        log(f"  failed request: {m}")
    return results, wall


def stream_stats(reqs, results, wall):
    """Latency = time from arrival to completion (the library's latency from
    submission plus the client's wait for buffer memory)."""
    idx = sorted(results)
    lat = np.array([results[i][0].latency_s + results[i][1] for i in idx])
    nrhs_done = sum(reqs[i][4] for i in results)
    big = [k for k, i in enumerate(idx) if reqs[i][1] == len(SERVE_SIZES) - 1]
    return {"requests": len(reqs), "completed": len(results),
            "all_ok": all(results[i][0].status == 0 for i in results),
            "status_counts": {str(k): int(v) for k, v in zip(*np.unique([results[i][0].status for i in idx],
                                                                        return_counts=True))},
            "p50_s": round(float(np.percentile(lat, 50)), 3), "p90_s": round(float(np.percentile(lat, 90)), 3),
            "p99_s": round(float(np.percentile(lat, 99)), 3), "max_s": round(float(lat.max()), 3),
            "mean_s": round(float(lat.mean()), 3), "wall_s": round(wall, 2),
            "requests_per_s": round(len(results) / wall, 4), "rhs_per_s": round(nrhs_done / wall, 3),
            "rhs": int(nrhs_done), "max_true_resid": max(results[i][0].true_resid for i in results),
            "max_client_wait_s": round(max(results[i][1] for i in results), 3),
            "p50_64x32_s": round(float(np.percentile(lat[big], 50)), 3) if big else None}


def serve_full(ctx, factors, nreq, nsat, sat_rate, inner_prec, max_rhs=12, seed=4242, nkv=32):
    """The serving workload at its stated scale: the saturation throughput is
    measured with a burst of nsat requests submitted at once (unless
    sat_rate is given), then streams of nreq Poisson requests arrive at each
    factor x saturation."""
    from paper_1710_08839_amd import qxd
    fields = serve_fields(ctx, inner_prec, nkv)
    s = qxd.solver(kind=qxd.SAP_GCR, tol=1e-10, nkv=nkv, ncy=4, nmr=4, inner_prec=inner_prec)
    out = {"inner_prec": PREC_NAME[inner_prec], "max_rhs": max_rhs,
           "workload": f"lattices {[f'{d[0]}x{d[1]}^3' for d in SERVE_SIZES]} (C*), q in {{2/3,-1/3}}, "
                       f"kappa~U[0.130,0.1365], csw=1.9, Gaussian or point sources, 1-{max_rhs} RHS, SAP-GCR "
                       f"(nkv {nkv}, ncy 4, nmr 4) to 1e-10"}
    rng = np.random.default_rng(seed)
    if sat_rate is None:
        reqs = draw_requests(rng, nsat, max_rhs, None)
        log(f"saturation burst of {nsat} requests")
        res, wall = run_stream(ctx, fields, reqs, s)
        out["saturation"] = stream_stats(reqs, res, wall)
        sat_rate = out["saturation"]["requests_per_s"]
        log(f"saturation: {out['saturation']}")
    out["saturation_requests_per_s"] = sat_rate
    for fct in factors:
        rate = fct * sat_rate
        reqs = draw_requests(rng, nreq, max_rhs, rate)
        log(f"stream at {fct} x saturation ({rate:.4f}/s), {nreq} requests")
        res, wall = run_stream(ctx, fields, reqs, s)
        out[f"stream_{fct}x"] = stream_stats(reqs, res, wall)
        out[f"stream_{fct}x"]["rate_per_s"] = round(rate, 4)
        log(f"stream {fct}x: {out[f'stream_{fct}x']}")
    for f in fields:
        f.release()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--nsrc", type=int, default=12, help="point sources per operator, batched solve leg")
    ap.add_argument("--nsrc-fp64", type=int, default=1, help="point sources per operator, FP64 baseline")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-single", action="store_true", help="skip the single right-hand-side solves")
    ap.add_argument("--serve-requests", type=int, default=12)
    ap.add_argument("--serve-max-rhs", type=int, default=3)
    ap.add_argument("--serve-rate", type=float, default=2.0, help="request arrivals per second")
    ap.add_argument("--precs", default="0,1,2,3")
    ap.add_argument("--dirac-variant", type=int, default=0,
                    help="force a Dirac kernel variant (0: autotune), e.g. to profile the tuned one")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 1 GiB device copy (profiler counter calibration)")
    ap.add_argument("--no-multishift", action="store_true")
    ap.add_argument("--no-sap", action="store_true")
    ap.add_argument("--no-dfl", action="store_true", help="skip the deflated SAP-GCR leg")
    ap.add_argument("--cpu-child", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--serve-full", action="store_true",
                    help="only the serving workload at its stated scale (saturation burst, then Poisson streams)")
    ap.add_argument("--serve-factors", default="0.8", help="arrival rates as fractions of saturation")
    ap.add_argument("--serve-sat", type=float, default=None, help="known saturation throughput (requests/s)")
    ap.add_argument("--serve-nsat", type=int, default=24, help="requests of the saturation burst")
    ap.add_argument("--serve-prec", default="f32")
    args = ap.parse_args()
    if args.cpu_child:
        # the CPU leg's own process: it never touches the GPU
        print(json.dumps(cpu_baseline_child(args.cpu_child)))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the library has no multi-GPU "
              f"path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1710_08839_amd import qxd, synth

    if args.serve_full:
        ctx = qxd.Context(0)
        res = serve_full(ctx, [float(x) for x in args.serve_factors.split(",")], args.serve_requests,
                         args.serve_nsat, args.serve_sat, qxd.PREC[args.serve_prec])
        ctx.close()
        print(json.dumps({"serve_full": res}))
        return

    dims = (64, 32, 32, 32)
    ctx = qxd.Context(0)
    if args.dirac_variant:
        qxd.set_dirac_variant(args.dirac_variant)
    t0 = time.perf_counter()
    log("generating the 64x32^3 gauge field")
    u, a = synth.gauge_field(dims, 20171002, 0.25, 0.15)
    field = qxd.Field(ctx, dims, u, a, cstar=3)
    log("field uploaded")
    del u, a
    q = qxd.quark(0.1365, -1 / 3, 1.9, 1.0)
    V = field.volume
    setup_s = time.perf_counter() - t0

    if args.copy_probe:
        # a plain device copy of known size (1 GiB read + 1 GiB written), for
        # calibrating the HBM byte counters of the profiler against the kernels
        a0 = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b0 = torch.empty_like(a0)
        b0.copy_(a0)
        torch.cuda.synchronize()
        del a0, b0

    precs = [int(p) for p in args.precs.split(",")]
    dw = {}
    for p in precs:
        # builds the operator in this precision before timing
        ms = time_applies(field, q, p, 3, 2, 1)
        ms = time_applies(field, q, p, 3, args.steps if p == 0 else max(10, args.steps // 2),
                          args.warmup)
        choice = args.dirac_variant or field.dirac_variant(p)
        gbs = site_bytes(p, choice) * V / (ms * 1e-3) / 1e9
        log(f"D {PREC_NAME[p]}: {ms:.4f} ms per application")
        dw[PREC_NAME[p]] = {"ms": round(ms, 4), "GB/s": round(gbs, 1),
                            "kernel": kernel_name(choice, p),
                            "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                            "GFLOP/s": round(FLOPS_PER_SITE * V / (ms * 1e-3) / 1e9, 1),
                            "bytes_per_site": site_bytes(p, choice)}

    # D at the sampled sites in every precision (API layout from the FP64
    # source), compared with the oracle after the timed legs
    sites = cfg2_sample_sites(V)
    x_dev = torch.from_numpy(synth.source(dims, 3, CFG2["src_seed"])).cuda()
    y_dev = torch.empty_like(x_dev)
    dw_at_sites = {}
    for p in precs:
        field.apply(q, qxd.OP_D, p, x_dev, y_dev)
        torch.cuda.synchronize()
        dw_at_sites[PREC_NAME[p]] = y_dev[torch.from_numpy(sites).cuda()].cpu().numpy()
    del x_dev, y_dev

    # the timed leg of the contract: K FP64 applications between barriers
    torch.cuda.synchronize()
    ms = time_applies(field, q, 0, 3, args.steps, args.warmup)
    choice = args.dirac_variant or field.dirac_variant(0)
    value = site_bytes(0, choice) * V / (ms * 1e-3) / 1e9
    kernel = kernel_name(choice, 0)
    stream_ceiling = {"read7_write1_GB/s": stream_gbs(7), "read5_write1_GB/s": stream_gbs(5),
                      "read6_write1_GB/s": stream_gbs(6), "copy_GB/s": stream_gbs(1),
                      "what": "library streaming probe: per thread 12 r 16-byte non-temporal loads folded "
                              "into 12 stores, 4 KB planes as in the block-major fields, 1 GiB written; "
                              "the FP64 D kernel reads 7 bytes per byte written, 5.5 with the mirror-fused "
                              "link reads"}
    log(f"streaming ceiling: {stream_ceiling}")

    multishift = None
    if not args.no_multishift:
        multishift = multishift_leg(field)
    sap = None if args.no_sap else sap_leg(field, q)
    single = None
    if not args.no_single:
        single = {"64x32^3": single_rhs_64x32(field)}
    deflation = None if args.no_dfl else dfl_leg(field)
    field.release()
    if single is not None:
        single["32x16^3"] = single_rhs_32x16(ctx)
        single["8x8^3"] = single_rhs_8x8(ctx)

    solves = None
    if not args.no_solve:
        solves = solve_rates(ctx, args.nsrc, args.nsrc_fp64)

    serve = None
    if not args.no_serve:
        serve = {}
        for name, prec in (("mixed_f32_inner", qxd.F32), ("fp64_inner", qxd.F64)):
            log(f"serving stream, {name}")
            serve[name] = serve_stream(ctx, args.serve_requests, args.serve_max_rhs, args.serve_rate, prec)
            log(f"serving {name}: p50 {serve[name]['p50_s']} s, p99 {serve[name]['p99_s']} s")

    ctx.close()
    cpu, dw_error = None, None
    if not args.no_cpu:
        log("timing the oracle on the host (child process)")
        cpu, expect = cpu_baseline_run()
        if expect is not None:
            dw_error = {k: float(np.linalg.norm(v - expect) / np.linalg.norm(expect))
                        for k, v in dw_at_sites.items()}
            dw_error["what"] = (f"|D_gpu - D_oracle| / |D_oracle| over {len(sites)} sampled sites of the "
                                f"64x32^3 C* lattice, FP64 source, autotuned kernels; bars 1e-12 (f64), "
                                f"1e-5 (f32), 1e-2 (f16s, bf16)")

    rec = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "Wilson-clover D (hop + Pauli), SU(3)xU(1), C* in x,y,z, "
                               "64x32^3 physical = 64x64x32x32 extended (4194304 sites), "
                               "q=-1/3, kappa=0.1365, csw=1.9, eps=0.25, A~N(0,0.15)",
                   "extended_sites": V, "rhs_per_application": 1, "gpus": 1},
        "roofline": {"bound": "hbm", "achieved": round(value, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(value / HBM_PEAK_GBS, 4), "traffic": TRAFFIC.get((kernel_hash(), choice)),
                     "kernel": kernel,
                     "bytes_per_launch": site_bytes(0, choice) * V},
        "dw": dw,
        "dw_error_vs_oracle": dw_error,
        "multishift": multishift,
        "sap": sap,
        "deflation": deflation,
        "stream_ceiling": stream_ceiling,
        "single_rhs": single,
        "solves": solves,
        "serve": serve,
        "cpu_baseline": cpu,
        "setup_s": round(setup_s, 1),
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
