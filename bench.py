"""Benchmark: flux-reconstruction Navier-Stokes RHS with flux anti-aliasing.

One step = one full right-hand-side evaluation (all kernel groups) of the
Taylor-Green vortex state on a 48^3 periodic hexahedral mesh, p = 3, with
6^3 Gauss-Legendre anti-aliasing points per element, fused kernels with
FP32 bulk arithmetic and FP64 state.  value = whole-job GDoF-RHS/s, with
DoF = 5 conserved variables x solution points (7.08M points, 35.4M DoF).
The same run reports the FP64 fused path and p = 4 alongside, the volume
kernel's HBM/ALU roofline position measured with HIP events, and the
reference oracle timed on the host on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GDoF-RHS/s NS+AA FR (fused FP32 vs plain FP64), % HBM roofline; p99 step ms"
HBM_PEAK_GBS = 8000.0
# published MI355X vector peaks: FP32 157.3 TFLOP/s (with packed FP32 math),
# FP64 78.6 TFLOP/s.  Without packed math the FP32 vector rate equals the
# FP64 one: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz = 78.6 TFLOP/s,
# reported beside it as the non-packed rate (this build emits no packed FP32).
VALU_PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}
VALU_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# HBM bytes per launch of the headline volume kernel (hex_volume<3, float> on
# the 48^3 workload), from two rocprofv3 --pmc runs (FETCH_SIZE x 2.000 +
# WRITE_SIZE x 1.000, factors from a 1 GiB copy), recorded in the profile
# summary of that kernel.  Valid for the kernel as profiled; None once the
# kernel changes.
HEX_VOL_P3_FP32_TRAFFIC = (286902 * 2 + 276480) * 1024

# FLOP counts of the point-wise physics (multiplies, adds and fused
# multiply-adds as 2; reciprocal and square root as 1), from the code of the
# device functions: the point flux f = f^e - f^v with the split energy
# component, the normal viscous flux, the interface flux of one own flux
# point (both sides' inviscid fluxes, Rusanov, LDG, the jump terms)
PF_FLOP, NV_FLOP, CF_FLOP = 147, 120, 140

NTYPE_PTS = {  # (N_u, flux points, quadrature points, faces) per element
    "hex": lambda n, m: (n ** 3, 6 * n * n, m ** 3, 6),
    "prism": lambda n, m: (n * n * (n + 1) // 2, n * (n + 1) + 3 * n * n, (n * n) * m, 5),
    "tet": lambda n, m: (n * (n + 1) * (n + 2) // 6, 2 * n * (n + 1), n ** 3, 4),
    "pyr": lambda n, m: (n * (n + 1) * (2 * n + 1) // 6, n * n + 2 * n * (n + 1), n ** 3, 5),
}


def volume_model(kind, p, prec, aa=True, diag=True):
    """Algorithmic HBM bytes and FLOPs of one element in the fused volume
    kernel, counted from the kernel's loops (not the MFMA tile padding).
    Bytes: state read (5 N_u doubles), neighbour face states (5 N_f reals,
    single precision with one float base per face and variable), normal
    viscous flux written (4 N_f reals), the four projected residual rows
    written and the mass-flux divergence L(rho v) read (N_u reals), face
    records, geometry and metrics.  FLOPs: the products of each phase
    (2 per multiply-add) and the point-wise physics (PF/NV_FLOP)."""
    rb = 4 if prec == "fp32" else 8
    n, m = p + 1, p + 3
    nu, nf, nq, nfc = NTYPE_PTS[kind](n, m)
    nvf = 4  # mass flux from L(rho v)
    byts = 5 * nu * 8 + 5 * nf * rb + 4 * nf * rb + nvf * nu * rb + nu * rb + nfc * (16 + 4 * rb) + 10 * rb
    if rb == 4:
        byts += nfc * 5 * 4
    S = 1 if diag else 3  # terms per transformed-flux component
    fl = 0
    if kind == "hex":
        fl += 3 * 5 * n * n * (4 * n + 4 + n * (2 * n + 3 + 1))   # face values, jumps, corrected gradient
        if not diag:
            fl += 5 * nu * 15                                       # J^-T
        fl += 3 * n * n * (80 * n + 2 * NV_FLOP)                   # face states + normal viscous flux
        if aa:
            fl += 40 * m * n ** 3                                   # x interpolation
            fl += m * m * 40 * n * n                                # y interpolation per column
            fl += m ** 3 * (40 * n + PF_FLOP + 3 * nvf * (2 * S - 1) + 3 * nvf * 2 * n)  # z, flux, z projection
            fl += nvf * m * n * n * 6 * m                           # y projection
            fl += nvf * n * n * n * 4 * m + 2 * n ** 3              # x projection, kap L
        else:
            fl += nu * (PF_FLOP + 3 * nvf * (2 * S - 1)) + nvf * nu * 3 * n * 2 + 2 * nu
    elif kind == "prism":
        nt, ntq = n * (n + 1) // 2, n * n
        fl += 5 * nt * (4 * n + 4) + 5 * n * 3 * n * (2 * nt + 2)  # face values and jumps
        fl += 5 * nt * n * (2 * n + 3) + 5 * n * nt * (4 * nt + 3 * (2 * n + 4))  # corrected gradient
        fl += 5 * nu * 15                                           # J^-T (general metric)
        fl += nt * (80 * n + 2 * NV_FLOP) + 3 * n * n * (40 * nt + NV_FLOP)  # face states + viscous flux
        if aa:
            fl += 20 * n * ntq * 2 * nt                              # triangle-plane interpolation
            fl += ntq * m * (40 * n + PF_FLOP + 3 * nvf * 5 + 3 * nvf * 2 * n)  # line columns
            fl += nvf * n * nt * 3 * ntq * 2 + 2 * nu                # triangle-plane projection, kap L
        else:
            fl += nu * (PF_FLOP + 3 * nvf * 5) + nvf * nu * 2 * (n + 2 * nt + 3 * n) + 2 * nu
    else:  # tetrahedra, pyramids: dense products
        fl += 2 * nf * nu * 5 + 5 * nf * 3                          # own face values, jumps
        fl += 2 * 3 * nu * (nu + nf) * 5 + 5 * nu * 15               # corrected gradient, J^-T
        fl += 2 * nf * nu * 20 + nf * NV_FLOP                       # face states + viscous flux
        if aa:
            fl += 2 * nq * nu * 20 + nq * (PF_FLOP + 3 * nvf * 6)     # quadrature values + flux
            fl += 2 * nu * 3 * nq * nvf + 2 * nu                      # projection-divergence, kap L
        else:
            fl += nu * (PF_FLOP + 3 * nvf * 6) + 2 * nu * 3 * nu * nvf + 2 * nu
    return byts, fl


def rhs_bytes_model(kind, p, prec):
    """Algorithmic bytes of one full fused RHS per element: disu reads U and
    writes U^f (+ face bases in single precision) and L(rho v); the volume
    group reads U, the neighbour U^f and L(rho v), writes V^f and the volume
    residual; the interface group reads the residual, own and neighbour U^f
    and V^f, and writes du.  Face records and metrics are not counted."""
    rb = 4 if prec == "fp32" else 8
    n, m = p + 1, p + 3
    nu, nf, _, nfc = NTYPE_PTS[kind](n, m)
    fb = nfc * 5 * 4 if rb == 4 else 0
    b = 5 * nu * 8 + 5 * nf * rb + fb + nu * rb
    b += 5 * nu * 8 + 5 * nf * rb + fb + nu * rb + 4 * nf * rb + 4 * nu * rb
    b += 5 * nu * rb + 2 * (5 * nf * rb + fb) + 2 * 4 * nf * rb + 5 * nu * 8
    return b


def plain_bytes_model(kind, p):
    """Algorithmic bytes per element of the plain FP64 path (every
    intermediate array in HBM, each written once and read once by the next
    kernel): W, U^f, C, Q~/Q, Q^f, U^q, Q^q/F~^q, R, D~."""
    n, m = p + 1, p + 3
    nu, nf, nq, _ = NTYPE_PTS[kind](n, m)
    w = 8
    b = 5 * nu * w * 2          # U read, W written
    b += 5 * nu * w + 5 * nf * w  # disu
    b += 2 * 5 * nf * w + 5 * nf * w  # con_u (own + neighbour read, C written)
    b += 5 * nu * w + 15 * nu * w + 5 * nf * w + 15 * nu * w  # tgradpcoru + tgradcoru
    b += 2 * 15 * nu * w        # gradcoru
    b += 15 * nu * w + 15 * nf * w  # gradcoru_fpts
    b += 15 * nu * w + 15 * nq * w + 5 * nu * w + 5 * nq * w  # gradcoru_qpts, qptsu
    b += 2 * 20 * nq * w         # tdisf (reads 20, writes 15; counted 20 + 20)
    b += 15 * nq * w + 5 * nu * w  # tdivtpcorf
    b += 2 * (5 + 15) * nf * w + 5 * nf * w  # comm_flux
    b += 5 * nf * w + 2 * 5 * nu * w  # tdivtconf
    b += 2 * 5 * nu * w          # negdivconf
    return b


def time_variant(frmi, torch, n, p, prec, steps, warmup, form="fused", kind="hex", aa=True, surface_aa=False):
    from paper_2401_06132_amd import inputs
    if form in ("noaa", "fullaa"):
        # the fused path without flux anti-aliasing (the paper's "AA off"), or
        # with flux and surface-flux anti-aliasing (its "full AA")
        aa, surface_aa, form = form == "fullaa", form == "fullaa", "fused"
    s = frmi.Solver(n, p, kind, prec=prec, pref=inputs.P0, rho_ref=inputs.RHO0, form=form, aa=aa, surface_aa=surface_aa)
    coords = s.upts_coords()
    U = inputs.element_state(coords, seed=0)
    u = torch.from_numpy(np.concatenate([x.reshape(-1) for x in U])).cuda()
    del U, coords
    du = torch.empty_like(u)
    for _ in range(warmup):
        s.rhs(u, du)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(steps):
        s.rhs(u, du)
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
    # dominant kernel (volume group) alone, same launch configuration
    vol_ms = float("nan")
    if form == "fused":
        for _ in range(max(1, warmup // 2)):
            s.rhs_stages(u, du, 2)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            s.rhs_stages(u, du, 2)
        e1.record()
        torch.cuda.synchronize()
        vol_ms = e0.elapsed_time(e1) / steps
    ok = bool(torch.isfinite(du).all().item())
    res = dict(n_dof=s.n_state, n_elem=s.n_hex + s.n_prism + s.n_tet + s.n_pyr, wall_s=wall, ms_per_step=wall * 1e3 / steps,
               p50_ms=float(np.percentile(per, 50)), p99_ms=float(np.percentile(per, 99)), vol_ms=vol_ms,
               finite=ok)
    del s, u, du
    torch.cuda.empty_cache()
    return res


def run_rk(frmi, torch, kind, n, p, prec, nsteps, dt):
    """nsteps RK4 steps on the internal state; per-step HIP-event times and
    the drift of the conserved integrals."""
    from paper_2401_06132_amd import inputs
    s = frmi.Solver(n, p, kind, prec=prec, pref=inputs.P0, rho_ref=inputs.RHO0)
    U = inputs.element_state(s.upts_coords(), seed=0)
    s.set_state(np.concatenate([x.reshape(-1) for x in U]))
    del U
    c0 = s.integrals()
    s.rk4(dt, 1)  # warm-up step (not timed), part of the trajectory
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(nsteps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(nsteps):
        s.rk4(dt, 1)
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(nsteps)])
    c1 = s.integrals()
    st = s.get_state()
    finite = bool(np.isfinite(st).all())
    vol = (2 * np.pi) ** 3
    # drift relative to the integral itself (mass, energy) or to the mass
    # integral (momentum, whose integral is ~0 for the vortex)
    scale = np.array([abs(c0[0]), abs(c0[0]), abs(c0[0]), abs(c0[0]), abs(c0[4])])
    out = dict(workload="Taylor-Green vortex, %d^3-cell periodic box, %s, p=%d, %s, %d RK4 steps of dt=%g"
               % (n, kind, p, prec, nsteps + 1, dt),
               elements=s.n_hex + s.n_prism + s.n_tet + s.n_pyr, n_hex=s.n_hex, n_prism=s.n_prism, dof=s.n_state,
               ms_per_step=wall * 1e3 / nsteps, p50_step_ms=float(np.percentile(per, 50)),
               p99_step_ms=float(np.percentile(per, 99)),
               gdof_rhs_s=s.n_state * 4 * nsteps / wall / 1e9, finite=finite,
               conservation_drift=[float(x) for x in (c1 - c0) / scale], domain_volume=vol)
    del s, st
    torch.cuda.empty_cache()
    return out


def serving_dt(n, p, kind, u0=1.0, c0=10.0):
    """RK4 step of a serving request: 0.25 h / ((2p+1)(U0 + c0)), h the cell
    size, c0 = 1/Ma (the same bound for hexahedra and prisms; twice this
    step is unstable on hexahedra)."""
    h = 2 * np.pi / n
    return 0.25 * h / ((2 * p + 1) * (u0 + c0))


def run_serving(frmi, torch, budget_gib=64.0, max_active=64, nreq=512, seed=0, check_every=64):
    """The serving stream: requests arrive by their Poisson schedule (wall
    clock), are queued, admitted by device footprint and slot limit, and
    advanced together one RK4 step per pool round until done.  Step latency
    = wall time of one pool round that advanced at least one request."""
    from paper_2401_06132_amd import inputs
    reqs = inputs.serving_requests(n=nreq, seed=seed)
    budget = int(budget_gib * (1 << 30))
    pool = frmi.Pool(budget, max_active=max_active, prec="fp32", pref=inputs.P0, rho_ref=inputs.RHO0)
    outs, t_arr, t_adm, t_fin, dof_req = {}, {}, {}, {}, {}
    step_ms, step_dof, active, launches = [], [], [], []
    peak_bytes, nxt, done, work = 0, 0, 0, 0
    t0 = time.perf_counter()
    last_print = t0
    while done < nreq:
        now = time.perf_counter() - t0
        while nxt < nreq and reqs[nxt]["arrival"] <= now:
            r = reqs[nxt]
            kw = dict(n=r["n"], p=r["p"], kind=r["etype"], nsteps=r["steps"],
                      dt=serving_dt(r["n"], r["p"], r["etype"]), tgv_p0=inputs.P0)
            if r["id"] % check_every == 0:
                kw["u_out"] = np.empty(pool.footprint(**kw)[1])
            rid = pool.submit(**kw)
            if "u_out" in kw:
                outs[rid] = kw["u_out"]
            t_arr[rid] = r["arrival"]
            dof_req[rid] = pool.footprint(**kw)[1]
            nxt += 1
        ts = time.perf_counter()
        st, adm, fin = pool.step()
        te = time.perf_counter()
        for i in adm:
            t_adm[i] = te - t0
        for i in fin:
            t_fin[i] = te - t0
        done += len(fin)
        peak_bytes = max(peak_bytes, st["bytes_in_use"])
        if st["n_active"] > 0:
            step_ms.append((te - ts) * 1e3)
            step_dof.append(st["dof"])
            active.append(st["n_active"])
            launches.append(st["n_launches"])
            work += 4 * st["dof"]
        elif st["n_queued"] == 0 and not adm and nxt < nreq:
            time.sleep(max(0.0, reqs[nxt]["arrival"] - (time.perf_counter() - t0)))
        if te - last_print > 10:
            last_print = te
            print("serving: t=%.1fs done=%d submitted=%d active=%d queued=%d" %
                  (te - t0, done, nxt, st["n_active"], st["n_queued"]), file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    lat = np.array([t_fin[i] - t_arr[i] for i in t_fin])
    wait = np.array([t_adm[i] - t_arr[i] for i in t_adm])
    finite = all(bool(np.isfinite(o).all()) for o in outs.values())
    sm = np.array(step_ms)
    return {
        "workload": "%d Taylor-Green requests, Poisson arrivals (mean %.0f/s), n^3 boxes n in 6..32, hex|prism, "
                    "p in {2,3,4}, 20-200 RK4 steps, fp32 fused" % (nreq, 200.0),
        "budget_GiB": budget_gib, "max_active": max_active, "requests": nreq, "wall_s": wall,
        "rounds": len(step_ms), "p50_step_ms": float(np.percentile(sm, 50)),
        "p99_step_ms": float(np.percentile(sm, 99)), "max_step_ms": float(sm.max()),
        "gdof_rhs_s": work / wall / 1e9, "gdof_rhs_s_busy": work / (sm.sum() * 1e-3) / 1e9,
        "mean_active": float(np.mean(active)), "max_active_seen": int(max(active)),
        "mean_launches_per_step": float(np.mean(launches)), "peak_GiB": peak_bytes / (1 << 30),
        "p50_request_latency_s": float(np.percentile(lat, 50)), "p99_request_latency_s": float(np.percentile(lat, 99)),
        "p50_queue_wait_s": float(np.percentile(wait, 50)), "p99_queue_wait_s": float(np.percentile(wait, 99)),
        "checked_finite": len(outs), "finite": finite,
    }


def cpu_baseline(budget_s=20.0):
    """The oracle (plain NumPy, dense operators) on the host: one RHS of the
    same Taylor-Green hex p=3 workload on a smaller periodic box; the box is
    chosen so that the run takes roughly budget_s seconds."""
    from oracle.mesh import Mesh
    from oracle.rhs import Params, rhs
    from paper_2401_06132_amd import inputs
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    def run(N):
        m = Mesh(N, N, N, 3, "hex")
        U = {t: u for t, u in zip(m.types, inputs.element_state([m.upts_coords(t) for t in m.types]))}
        t0 = time.perf_counter()
        rhs(m, U, Params(pref=inputs.P0))
        return time.perf_counter() - t0, 5 * m.nelem["hex"] * m.refs["hex"].nu

    # an 8^3 probe sizes the sample box for about budget_s of work
    t8, _ = run(8)
    N = int(max(8, min(32, round(8 * (budget_s / max(t8, 1e-3)) ** (1.0 / 3.0)))))
    elapsed, dof = run(N)
    return {"value": dof / elapsed / 1e9, "unit": "GDoF-RHS/s", "cores": int(threads), "kind": "oracle",
            "sample": "one RHS of the TGV hex p=3 flux-AA case on a %d^3 periodic box (%d DoF), %.2f s" %
                      (N, dof, elapsed)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=48)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline variant only")
    ap.add_argument("--only", default=None, help="one variant kind:prec:p:form, e.g. prism:fp32:3:fused (profiling)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving stream")
    ap.add_argument("--serving-only", action="store_true", help="only the serving stream")
    ap.add_argument("--serving-budget-gib", type=float, default=64.0)
    ap.add_argument("--serving-slots", type=int, default=64)
    ap.add_argument("--serving-requests", type=int, default=512)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device-to-device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (see DESIGN.md, sharding)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2401_06132_amd as frmi
    torch.cuda.set_device(0)
    if args.copy_probe:
        # a 1 GiB device-to-device copy: calibrates the HBM byte counters and
        # gives the copy bandwidth (bytes read + written per second), the
        # practical ceiling of a streaming kernel
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(10):
            dst.copy_(src)
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / 10
        nb = src.numel() * 4
        print(json.dumps({"copy_probe_bytes_each_way": nb, "copies": 13, "ms_per_copy": round(ms, 4),
                          "copy_GBs": round(2 * nb / (ms * 1e-3) / 1e9, 1)}))
        return
    if args.serving_only:
        sv = run_serving(frmi, torch, args.serving_budget_gib, args.serving_slots, args.serving_requests)
        print(json.dumps({"serving": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in sv.items()}}),
              flush=True)
        return
    variants = {}
    if args.only:
        kind, prec, p, form = args.only.split(":")
        r = time_variant(frmi, torch, args.n, int(p), prec, args.steps, args.warmup, form, kind)
        r["gdof_s"] = r["n_dof"] * args.steps / r["wall_s"] / 1e9
        if kind in NTYPE_PTS and form in ("fused", "noaa"):
            vb, vf = volume_model(kind, int(p), prec, aa=form == "fused")
            r["vol_TFLOPs"] = vf * r["n_elem"] / (r["vol_ms"] * 1e-3) / 1e12
            r["vol_GBs"] = vb * r["n_elem"] / (r["vol_ms"] * 1e-3) / 1e9
        print(json.dumps({"variant": args.only, **{k: (round(v, 4) if isinstance(v, float) else v)
                                                   for k, v in r.items()}}), flush=True)
        return
    order = [("fp32", 3, "fused", "hex")] if args.quick else [
        ("fp32", 3, "fused", "hex"), ("fp64", 3, "fused", "hex"), ("fp64", 3, "plain", "hex"),
        ("fp32", 4, "fused", "hex"), ("fp64", 4, "fused", "hex"), ("fp64", 4, "plain", "hex"),
        ("fp32", 3, "fused", "prism"), ("fp64", 3, "fused", "prism"), ("fp64", 3, "plain", "prism"),
        ("fp32", 4, "fused", "prism"), ("fp64", 4, "fused", "prism"), ("fp64", 4, "plain", "prism"),
        ("fp32", 3, "noaa", "hex"), ("fp64", 3, "noaa", "hex"), ("fp32", 4, "noaa", "hex"),
        ("fp32", 3, "noaa", "prism"), ("fp32", 4, "noaa", "prism"),
        ("fp32", 3, "fullaa", "hex"), ("fp64", 3, "fullaa", "hex"), ("fp32", 4, "fullaa", "hex"),
        ("fp64", 4, "fullaa", "hex"), ("fp32", 3, "fullaa", "prism"), ("fp32", 4, "fullaa", "prism"),
        ("fp32", 3, "fused", "tet"), ("fp64", 3, "fused", "tet"), ("fp32", 4, "fused", "tet"),
        ("fp32", 3, "noaa", "tet"), ("fp32", 4, "noaa", "tet"), ("fp64", 3, "plain", "tet"),
        ("fp32", 3, "fused", "pyr"), ("fp64", 3, "fused", "pyr"), ("fp32", 4, "fused", "pyr"),
        ("fp32", 3, "noaa", "pyr"), ("fp64", 3, "plain", "pyr"), ("fp32", 3, "fused", "hex_pyr"),
        ("fp32", 3, "fused", "hex_pyr_tet"), ("fp32", 3, "fused", "hex_prism_pyr_tet"),
        ("fp32", 3, "fused", "hex_warp"), ("fp64", 3, "fused", "hex_warp"), ("fp32", 4, "fused", "hex_warp"),
        ("fp32", 3, "fused", "prism_warp"), ("fp32", 4, "fused", "prism_warp")]
    for prec, p, form, kind in order:
        ksteps = args.steps if kind == "hex" else max(5, args.steps // 3)
        r = time_variant(frmi, torch, args.n, p, prec, ksteps, args.warmup, form, kind)
        E = r["n_elem"]
        r["gdof_s"] = r["n_dof"] * ksteps / r["wall_s"] / 1e9
        r["vol_GBs"] = r["vol_TFLOPs"] = r["vol_frac"] = r["rhs_GBs"] = float("nan")
        if kind in NTYPE_PTS:
            # single-type affine meshes: the volume kernel's position against
            # its roof, and the whole RHS against HBM
            if form in ("fused", "noaa"):
                vb, vf = volume_model(kind, p, prec, aa=form == "fused")
                r["vol_GBs"] = vb * E / (r["vol_ms"] * 1e-3) / 1e9
                r["vol_TFLOPs"] = vf * E / (r["vol_ms"] * 1e-3) / 1e12
                r["vol_frac"] = r["vol_TFLOPs"] / VALU_PEAK_TFLOPS[prec]
            if form in ("fused", "noaa", "fullaa"):
                r["rhs_GBs"] = rhs_bytes_model(kind, p, prec) * E * ksteps / r["wall_s"] / 1e9
            elif form == "plain":
                r["rhs_GBs"] = plain_bytes_model(kind, p) * E * ksteps / r["wall_s"] / 1e9
        variants["%s%s%s_p%d" % ("" if kind == "hex" else kind + "_", "" if form == "fused" else form + "_", prec,
                                  p)] = r
        print("variant", kind, form, prec, p,
              json.dumps({k: round(v, 4) if isinstance(v, float) else v for k, v in r.items()}),
              file=sys.stderr, flush=True)
    head = variants["fp32_p3"]
    for pre in ("", "prism_", "tet_", "pyr_"):
        for p in (3, 4):
            a, b = "%sfp32_p%d" % (pre, p), "%splain_fp64_p%d" % (pre, p)
            if a in variants and b in variants:
                variants[a]["speedup_vs_plain_fp64"] = variants[a]["gdof_s"] / variants[b]["gdof_s"]
    vb, vf = volume_model("hex", 3, "fp32")
    ai = vf / vb
    peak = VALU_PEAK_TFLOPS["fp32"]
    ridge = peak * 1e12 / (HBM_PEAK_GBS * 1e9)
    if ai > ridge:
        roof = {"bound": "alu", "achieved": round(head["vol_TFLOPs"], 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(head["vol_TFLOPs"] / peak, 4),
                "peak_nonpacked": round(VALU_NONPACKED_TFLOPS, 1),
                "frac_nonpacked": round(head["vol_TFLOPs"] / VALU_NONPACKED_TFLOPS, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(head["vol_GBs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(head["vol_GBs"] / HBM_PEAK_GBS, 4)}
    traffic = HEX_VOL_P3_FP32_TRAFFIC if args.n == 48 else None
    roof.update({"traffic": traffic, "kernel": "hex_volume<3,float> (diagonal metric)",
                 "traffic_unit": "bytes per launch", "flop_per_elem": vf, "bytes_per_elem": vb,
                 "algorithmic_bytes": vb * head["n_elem"], "hbm_GBs": round(head["vol_GBs"], 1),
                 "hbm_frac": round(head["vol_GBs"] / HBM_PEAK_GBS, 4), "flop_per_byte": round(ai, 2),
                 "avg_ms": round(head["vol_ms"], 4)})
    def _r(x):
        return round(x, 4) if isinstance(x, float) and np.isfinite(x) else (x if not isinstance(x, float) else None)
    out = {
        "metric": METRIC, "value": round(head["gdof_s"], 3), "unit": "GDoF-RHS/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "Taylor-Green vortex, %d^3 periodic hex, p=3, flux AA GL(6)^3, fused, FP32 bulk / "
                               "FP64 state" % args.n, "elements": head["n_elem"], "dof": head["n_dof"]},
        "p50_step_ms": round(head["p50_ms"], 4), "p99_step_ms": round(head["p99_ms"], 4),
        "hbm_frac_rhs": round(head["rhs_GBs"] / HBM_PEAK_GBS, 4),
        "roofline": roof,
        "variants": {k: {"gdof_s": _r(v["gdof_s"]), "p99_step_ms": _r(v["p99_ms"]), "vol_ms": _r(v["vol_ms"]),
                         "vol_TFLOPs": _r(v["vol_TFLOPs"]), "vol_GBs": _r(v["vol_GBs"]),
                         "vol_frac": _r(v["vol_frac"]), "hbm_frac_rhs": _r(v["rhs_GBs"] / HBM_PEAK_GBS),
                         "finite": v["finite"],
                         "speedup_vs_plain_fp64": _r(v.get("speedup_vs_plain_fp64", float("nan")))}
                     for k, v in variants.items()},
    }
    if not args.quick:
        rk = run_rk(frmi, torch, "mixed", 64, 4, "fp32", 99, 2e-4)
        out["mixed_rk4"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in rk.items()}
        print("mixed rk4", json.dumps(out["mixed_rk4"]), file=sys.stderr, flush=True)
    if not args.quick and not args.no_serving:
        sv = run_serving(frmi, torch, args.serving_budget_gib, args.serving_slots, args.serving_requests)
        out["serving"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in sv.items()}
        print("serving", json.dumps(out["serving"]), file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
