"""Benchmark: MAC solves per second to a 1e-10 relative residual on one MI355X.

One step = one whole MAC projection as a time step of the method performs it
(Sec. 3.2 Steps 3/7): map the base state to face coefficients (fill + harmonic
faces + coefficient hierarchy), assemble the right-hand side, solve to
||r||/||b|| <= 1e-10, and correct the face velocity, on device-resident inputs
of the 256^3 plane-parallel workload (periodic x/y, Neumann z, 1e4 density
contrast, seeded).  `value` is the mixed-precision rate (FP32 V(2,2) cycles in
FP64 iterative refinement); the plain FP64 V-cycle rate is reported beside it.

The JSON line also carries the roofline of the dominant kernel (the finest-
level smoother, timed per launch with HIP events on the library's stream),
the FP64 CPU oracle timed on the host for a bounded sample, and:
  workloads  the same measurement on the 512^3 plane-parallel (1e5 contrast)
             and 384^3 spherical star workloads, whose smoother working sets
             (1.6 GB and 0.7 GB per sweep) exceed the 256 MB Infinity Cache,
             with the phi error of the 512^3 solve against the FP64 oracle's
             (--no-large skips them, --no-oracle-error the oracle solve);
  adjoint    forward + backward of the differentiable solve (autograd
             function: solve, adjoint solve, coefficient gradient) on the
             128^3 FP64 and 512^3 mixed workloads (--no-adjoint);
  nodal      the nodal projection (Sec. 3.2 Step 11) on the same base state
             with a cell-centred velocity (--no-nodal);
  base1d     with --base1d: Enforce HSE, beta0 and w0 on the irregular radii
             of 256^3 and 1536^3 boxes.
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

PEAK_HBM_GBS = 8000.0
METRIC = "MAC solves/sec to 1e-10 residual (mixed vs FP64) + stencil HBM GB/s"
WORKLOAD = "c2"
LARGE = ("c5", "c3")


def _parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=WORKLOAD, choices=["c1", "c2", "c3", "c5"])
    ap.add_argument("--fp64-steps", type=int, default=None, help="steps of the FP64 comparison (default: steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=1, help="oracle projections timed on the host")
    ap.add_argument("--only", choices=["mixed", "fp64"], default=None, help="time one precision only")
    ap.add_argument("--no-nodal", action="store_true", help="skip the nodal-projection timing")
    ap.add_argument("--nodal-steps", type=int, default=10)
    ap.add_argument("--no-large", action="store_true", help="skip the 512^3 and 384^3 workloads")
    ap.add_argument("--large-steps", type=int, default=5)
    ap.add_argument("--no-oracle-error", action="store_true",
                    help="skip the FP64 oracle solve of the 512^3 workload (phi error)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the forward + backward timing")
    ap.add_argument("--adjoint-steps", type=int, default=5)
    ap.add_argument("--base1d", action="store_true", help="time Enforce HSE, beta0 and w0 on irregular radii")
    ap.add_argument("--smoother", choices=["auto", "per_colour"], default="auto",
                    help="per_colour: one launch per colour on every level (the default runs both colours of a "
                         "finest-level sweep in one launch where rows are 128 to 512 cells)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 256 MiB streaming copy (reference for the HBM traffic counters)")
    return ap.parse_args()


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _traffic_record(key):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f).get(key)
    except (OSError, ValueError):
        return None
    if not rec:
        return None
    # the counters belong to the kernel source they were taken on
    import hashlib

    # (the .hip file and the headers it includes, hashed in the listed order)
    h = hashlib.sha256()
    for rel in rec.get("sources", []):
        src = os.path.join(ROOT, rel)
        if not os.path.exists(src):
            return None
        with open(src, "rb") as f:
            h.update(f.read())
    if not rec.get("sources") or h.hexdigest() != rec.get("sha256"):
        return None
    return rec


def _describe(p):
    bcs = "".join("PN"[b] for b in p.bc)
    if p.geometry == 0:
        shape = f"plane-parallel exponential atmosphere, {p.meta.get('contrast'):.0e} density contrast"
    else:
        shape = f"spherical star (linear radial fill at dr = h/5), {p.meta.get('contrast'):.0e} contrast to the box face"
    return f"{p.nx}x{p.ny}x{p.nz} {shape}, boundaries (x,y,z) {bcs}"


def _tensors(p, dev):
    import numpy as np
    import torch

    def T(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    return T(p.beta0_1d), T(p.rho), T(p.S), [T(p.ux), T(p.uy), T(p.uz)]


def _time_projection(p, dev, precision, steps, warmup, smoother="auto", keep_phi=False):
    """Whole projections (map + rhs + solve to 1e-10 + correction) on
    device-resident inputs; returns (seconds for `steps`, infos, phi)."""
    import torch

    from paper_1908_03634_amd import mproj

    beta0_1d, rho, S, U0 = _tensors(p, dev)
    ctx = mproj.Context(p.nx, p.ny, p.nz, h=p.h, bc=p.bc, precision=precision, rtol=1e-10, smoother=smoother)
    total = steps + warmup
    # every step projects its own copy of the unprojected velocity
    copies = [[u.clone() for u in U0] for _ in range(total)]
    phi = ctx.empty_cells()
    infos = []
    torch.cuda.synchronize()
    t0 = None
    for s in range(total):
        if s == warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        # the last timed step also timestamps each finest-level smoother
        # launch (the roofline sample); the others run uninstrumented
        ctx.set_kernel_timing(s == total - 1)
        ctx.map_base_state(p.geometry, beta0_1d, rho, p.dr, p.center, want_coefs=False)
        _, info = ctx.mac_project(*copies[s], S, phi=phi)
        if s >= warmup:
            infos.append(info)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    del copies
    out_phi = phi if keep_phi else None
    return dt, infos, out_phi


def _roofline(workload, infos, precision):
    """Roofline of the finest-level smoother from the per-launch HIP-event
    timestamps of the last timed step: algorithmic bytes per launch (x read
    unless from a zero start, x written, b and the cell coefficients read, one
    word each per cell; 1/8 word of coarse correction after prolongation; 16
    bytes per cell where the refinement update rides on the launch) divided by
    the launch-weighted average duration."""
    tot_ms = sum(i["smooth_ms_total"] for i in infos)
    cnt = sum(i["smooth_launches"] for i in infos)
    tot_bytes = sum(i["smooth_bytes"] for i in infos)
    avg_s = tot_ms / cnt / 1e3 if cnt else float("nan")
    bytes_per_launch = tot_bytes / cnt if cnt else float("nan")
    achieved = bytes_per_launch / avg_s / 1e9
    if precision == "mixed":
        kname = "k_fsw_lds<float>" if infos[-1].get("smooth_form") == 1 else "k_gs_blk<float>"
    else:
        kname = "k_gs_blk<double>"
    rec = _traffic_record(f"{workload}:{kname}")
    traffic = None
    if rec:
        # HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE counters,
        # averaged over the same launches as `achieved` and scaled by the
        # counters' reading of the calibration copy
        traffic = {"fetch_bytes": rec["fetch_bytes"], "write_bytes": rec["write_bytes"],
                   "total_bytes": rec["fetch_bytes"] + rec["write_bytes"],
                   "algorithmic_bytes": rec.get("algorithmic_bytes"), "calibration": rec.get("calibration"),
                   "summary": rec.get("summary")}
    return {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic["total_bytes"] if traffic else None, "traffic_detail": traffic,
            "avg_launch_us": round(avg_s * 1e6, 2), "launches": cnt,
            "bytes_per_launch": round(bytes_per_launch)}


def _large(name, args, dev):
    """Mixed and FP64 rates, the smoother's roofline and (512^3) the phi error
    against the FP64 oracle on one of the workloads larger than the cache."""
    import numpy as np

    from paper_1908_03634_amd import workloads as W

    p = W.config_problem(name)
    _log(f"workload {p.name}: {p.nx}x{p.ny}x{p.nz}, bc {p.bc}")
    K, Wm = args.large_steps, 2
    mdt, minfos, phi = _time_projection(p, dev, "mixed", K, Wm, keep_phi=(name == "c5"))
    fdt, finfos, _ = _time_projection(p, dev, "fp64", K, Wm)
    last = minfos[-1]
    out = {"workload": f"{name}: {_describe(p)}", "value": round(K / mdt, 3), "unit": "solves/s",
           "ms_per_step": round(1e3 * mdt / K, 4), "steps": K, "fp64_value": round(K / fdt, 3),
           "fp64_ms_per_step": round(1e3 * fdt / K, 4), "mixed_over_fp64": round(fdt / mdt, 3),
           "outer_steps": last["outer_iters"], "vcycles": last["vcycles"], "rel_resid": last["rel_resid"],
           "bottom_iters": last["bottom_iters_total"], "levels": last["levels"],
           "phase_ms": {"setup": round(last["ms_setup"], 4), "rhs": round(last["ms_rhs"], 4),
                        "solve": round(last["ms_solve"], 4), "correct": round(last["ms_correct"], 4)},
           "roofline": _roofline(name, minfos, "mixed")}
    _log(f"{name}: mixed {out['value']} solves/s, fp64 {out['fp64_value']}, smoother "
         f"{out['roofline']['achieved']} GB/s ({out['roofline']['frac']})")
    if phi is not None and not args.no_oracle_error:
        import oracle

        oracle.build(force=False)
        t0 = time.perf_counter()
        ref = oracle.mac_project(p, tol=1e-12)
        err = float(np.linalg.norm(phi.cpu().numpy() - ref["phi"]) / np.linalg.norm(ref["phi"]))
        out["phi_error_vs_oracle"] = {"value": err, "gpu_rtol": 1e-10, "oracle_rtol": 1e-12,
                                      "oracle_seconds": round(time.perf_counter() - t0, 1),
                                      "rel_resid": out.get("rel_resid"),
                                      "note": "relative L2 error of the benchmarked mixed solve's phi; it follows "
                                              "the residual the solve stops at (at most the condition number times "
                                              "it); solved to 1e-12 the tests hold phi within 1e-9"}
        _log(f"{name}: phi error vs the oracle {err:.3e}")
    return out


def _adjoint(name, precision, args, dev):
    """Forward + backward through the autograd function (phi = solve(rhs; c),
    L = <w, phi>): the forward solve, the adjoint solve and the coefficient
    gradient per step, the coefficients loaded once (the same tensors every
    step), inputs on the device."""
    import numpy as np
    import torch

    from paper_1908_03634_amd import mproj, workloads as W
    from paper_1908_03634_amd.autograd import mac_solve

    p = W.config_problem(name)

    def T(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    ctx = mproj.Context(p.nx, p.ny, p.nz, h=p.h, bc=p.bc, precision=precision, rtol=1e-10)
    cx, cy, cz = ctx.map_base_state(p.geometry, T(p.beta0_1d), T(p.rho), p.dr, p.center)
    ux, uy, uz = T(p.ux), T(p.uy), T(p.uz)
    # the solve input: the projection's right-hand side (div(beta0 U) - beta0 S)
    phi0, _ = ctx.mac_project(ux, uy, uz, T(p.S))
    rhs = ctx.apply(phi0)
    del ux, uy, uz, phi0
    cs = [c.clone().requires_grad_(True) for c in (cx, cy, cz)]
    w = T(p.w)
    K, Wm = args.adjoint_steps, 1
    torch.cuda.synchronize()
    t0 = None
    for s in range(K + Wm):
        if s == Wm:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        ctx.set_kernel_timing(s == K + Wm - 1)
        r = rhs.detach().requires_grad_(True)
        phi = mac_solve(ctx, r, *cs)
        (phi * w).sum().backward()
        for c in cs:
            c.grad = None
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    out = {"workload": f"{name}: {_describe(p)}", "precision": precision, "value": round(K / dt, 3),
           "unit": "forward+backward/s", "ms_per_step": round(1e3 * dt / K, 4), "steps": K,
           "note": "per step: forward solve, adjoint solve, face-coefficient gradient (G lam)(G phi); "
                   "face coefficients on every level (stored faces on the finest)"}
    _log(f"adjoint {name} {precision}: {out['value']} forward+backward/s")
    return out


def _base1d(dev):
    """Enforce HSE, beta0 and w0 on the irregular radii of 256^3 and 1536^3
    boxes (20 calls each, the host waiting at the end)."""
    import numpy as np
    import torch

    import oracle
    from paper_1908_03634_amd import mproj

    oracle.build(force=False)
    ctx = mproj.Context(16, 16, 16, bc=(1, 1, 1), precision="fp64")
    out = {}
    for n in (256, 1536):
        nm = oracle.radius_count(n, n, n)
        rc, re = oracle.irregular_radii(nm, 1.0 / n)
        rho0 = (1.0 + (rc / 0.05) ** 2) ** -2.5
        g = 1.0 / (0.01 + re ** 2)

        def d(a):
            return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

        trc, tre, trho, tg = d(rc), d(re), d(rho0), d(g)
        gam = d(np.full(nm, 5 / 3))
        sbar = d(np.sin(rc * 20))
        p0, _ = ctx.enforce_hse(trc, trho, tg, 10.0, 1e-5)
        b = ctx.beta0_from_p0(rho0[0], p0, gam)
        w = ctx.w0(2, trc, tre, b, sbar)
        torch.cuda.synchronize()
        rec = {"radii": nm}
        for name, f in (("enforce_hse_us", lambda: ctx.enforce_hse(trc, trho, tg, 10.0, 1e-5, out=p0)),
                        ("beta0_us", lambda: ctx.beta0_from_p0(rho0[0], p0, gam, out=b)),
                        ("w0_us", lambda: ctx.w0(2, trc, tre, b, sbar, out=w))):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(20):
                f()
            torch.cuda.synchronize()
            rec[name] = round(1e6 * (time.perf_counter() - t0) / 20, 1)
        t0 = time.perf_counter()
        op0, _ = oracle.enforce_hse(rc, rho0, g, 10.0, 1e-5)
        oracle.beta0_from_p0(rho0[0], op0, np.full(nm, 5 / 3))
        rec["oracle_hse_beta0_ms"] = round(1e3 * (time.perf_counter() - t0), 2)
        out[f"{n}^3"] = rec
        _log(f"base1d {n}^3 ({nm} radii): {rec}")
    ctx.close()
    # the lateral Average of a cell field over the radii of a star (the
    # device-built octant list, then the fold and per-radius sums per call)
    for n in (256, 512):
        c2 = mproj.Context(n, n, n, bc=(1, 1, 1), precision="fp64")
        nm = c2.radius_count()
        phi = torch.randn((n, n, n), dtype=torch.float64, device=dev)
        avg = torch.empty(nm, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c2.average(phi, out=avg, count=False)
        torch.cuda.synchronize()
        first = time.perf_counter() - t0
        t0 = time.perf_counter()
        for _ in range(20):
            c2.average(phi, out=avg, count=False)
        torch.cuda.synchronize()
        per = (time.perf_counter() - t0) / 20
        n1d = int(np.ceil(5 * np.sqrt(3.0) * n / 2)) + 2
        avu = torch.empty(n1d, dtype=torch.float64, device=dev)
        t0 = time.perf_counter()
        for _ in range(20):
            c2.average_uniform(phi, n1d, 1.0 / (5 * n), out=avu)
        torch.cuda.synchronize()
        peru = (time.perf_counter() - t0) / 20
        rec = {"radii": nm, "first_call_ms": round(1e3 * first, 2), "average_us": round(1e6 * per, 1),
               "average_GBps": round(8.0 * n ** 3 / per / 1e9, 1), "uniform_average_us": round(1e6 * peru, 1)}
        out[f"average {n}^3"] = rec
        _log(f"average {n}^3: {rec}")
        c2.close()
        del phi
    return out


def main():
    args = _parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the solve is not sharded across GPUs",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch

    from paper_1908_03634_amd import workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(1)
    dev = torch.device("cuda:0")
    p = W.config_problem(args.workload)
    _log(f"workload {p.name}: {p.nx}x{p.ny}x{p.nz}, bc {p.bc}")
    K, Wm = args.steps, args.warmup

    if args.copy_calibration:
        # a streaming kernel of known traffic (reads and writes 256 MiB each;
        # an elementwise product, so its name differs from every copy the
        # benchmark makes) to scale the HBM counters of the other kernels
        nbytes = 256 << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        _log(f"copy calibration: 3 elementwise copies reading and writing {nbytes} bytes each")
        del src, dst

    res = {}
    for prec in ("mixed", "fp64"):
        if args.only and prec != args.only:
            continue
        steps = K if prec == "mixed" else (args.fp64_steps or K)
        dt, infos, _ = _time_projection(p, dev, prec, steps, Wm, smoother=args.smoother)
        res[prec] = (dt, steps, infos)
        _log(f"{prec}: {steps / dt:.2f} solves/s, {1e3 * dt / steps:.3f} ms/step, "
             f"steps {infos[-1]['outer_iters']}, rel {infos[-1]['rel_resid']:.2e}")

    main_prec = args.only or "mixed"
    dt, steps, infos = res[main_prec]
    value = steps / dt
    roofline = _roofline(args.workload, infos, main_prec)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        oracle.build(force=False)
        t0 = time.perf_counter()
        for _ in range(args.cpu_samples):
            r = oracle.mac_project(p, tol=1e-10)
        cdt = time.perf_counter() - t0
        cpu = {"value": round(args.cpu_samples / cdt, 4), "unit": "solves/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"{args.cpu_samples} full {p.nx}x{p.ny}x{p.nz} projection(s) (fill, faces, rhs, FP64 "
                         f"V(2,2) multigrid to 1e-10 in {r['info']['cycles']} cycles, correction)"}
        _log(f"cpu oracle: {cpu['value']} solves/s on {cpu['cores']} threads")

    last = infos[-1]
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": Wm,
        "ms_per_step": round(1e3 * dt / steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if main_prec == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {_describe(p)}; map + rhs + solve to 1e-10 + "
                               f"velocity correction per step",
                   "precision": main_prec, "smoother": "red-black Gauss-Seidel V(2,2)",
                   "outer_steps": last["outer_iters"], "vcycles": last["vcycles"], "rel_resid": last["rel_resid"],
                   "bottom_iters": last["bottom_iters_total"], "levels": last["levels"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if "fp64" in res and main_prec != "fp64":
        fdt, fsteps, finfos = res["fp64"]
        line["fp64_value"] = round(fsteps / fdt, 3)
        line["fp64_ms_per_step"] = round(1e3 * fdt / fsteps, 4)
        line["fp64_cycles"] = finfos[-1]["vcycles"]
        line["mixed_over_fp64"] = round(value / (fsteps / fdt), 3)
    line["phase_ms"] = {"setup": round(last["ms_setup"], 4), "rhs": round(last["ms_rhs"], 4),
                        "solve": round(last["ms_solve"], 4), "correct": round(last["ms_correct"], 4)}
    if not args.no_large:
        line["workloads"] = {name: _large(name, args, dev) for name in LARGE if name != args.workload}
    if not args.no_adjoint:
        line["adjoint"] = {"c4": _adjoint("c4", "fp64", args, dev), "c5": _adjoint("c5", "mixed", args, dev)}
    if not args.no_nodal:
        line["nodal"] = _nodal(args, dev)
    if args.base1d:
        line["base1d"] = _base1d(dev)
    print(json.dumps(line), flush=True)


def _nodal(args, dev):
    """The nodal projection of Sec. 3.2 Step 11 on the same base state with a
    cell-centred velocity: map + right-hand side + solve to 1e-10 + velocity
    correction per step, mixed precision."""
    import numpy as np
    import torch

    from paper_1908_03634_amd import mproj, workloads as W

    p = W.config_problem(args.workload, velocity="cells")

    def T(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    beta0_1d, rho, S = T(p.beta0_1d), T(p.rho), T(p.S)
    U0 = [T(p.ux), T(p.uy), T(p.uz)]
    ctx = mproj.Context(p.nx, p.ny, p.nz, h=p.h, bc=p.bc, precision="mixed", rtol=1e-10)
    phi = ctx.empty_nodes()
    warm, steps = 2, args.nodal_steps
    U = [u.clone() for u in U0]
    info = None
    torch.cuda.synchronize()
    t0 = None
    for s in range(warm + steps):
        if s == warm:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        for u, u0 in zip(U, U0):
            u.copy_(u0)
        ctx.map_base_state(p.geometry, beta0_1d, rho, p.dr, p.center, want_coefs=False)
        _, info = ctx.nodal_project(*U, S, phi=phi)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    out = {"workload": f"{args.workload} with cell-centred velocity: {_describe(p)}; nodes "
                       f"{'x'.join(str(m) for m in reversed(tuple(phi.shape)))}",
           "value": round(steps / dt, 3), "unit": "projections/s", "ms_per_step": round(1e3 * dt / steps, 4),
           "steps": steps, "precision": "mixed", "smoother": "4-colour Gauss-Seidel V(2,2)",
           "outer_steps": info["outer_iters"], "vcycles": info["vcycles"], "rel_resid": info["rel_resid"],
           "div_defect": round(info["div_defect"], 4),
           "phase_ms": {"rhs": round(info["ms_rhs"], 4), "solve": round(info["ms_solve"], 4),
                        "correct": round(info["ms_correct"], 4)},
           "note": "includes a device copy of the three unprojected velocity arrays per step"}
    _log(f"nodal: {out['value']} projections/s, {out['ms_per_step']} ms/step")
    return out


if __name__ == "__main__":
    main()
