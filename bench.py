"""Benchmark: fast-multipole BEM matrix-vector product and solve on one MI355X.

Workload (default): Laplace, unit sphere of 20480 curved 6-node triangles
(40962 collocation nodes), point-source Neumann data, order-8 expansions,
at most 48 elements per leaf, separation factor 0.62.  A step is one application of the system
operator A x = c.x - K x through the fast product (strengths, P2M, M2M, M2L,
L2L, L2P, near field, corrections and free term), with the input already in
device memory.  The headline value is the mixed-precision product
(single-precision near field and expansions, double corrections); the plain
FP64 product, both GMRES(50) solves to a 1e-8 residual, errors against the
oracle, per-phase device times and the dominant kernel's roofline are
reported beside it.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sphere20480] [--no-cpu]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP32_VEC_PEAK = 157.3  # TFLOP/s, MI355X vector FP32 (256 CUs, 2.4 GHz, packed)
FP32_MFMA_PEAK = 157.3  # TFLOP/s, MI355X dense FP32 matrix
FP64_VEC_PEAK = 78.6
KERNEL_PEAKS = {"m2l": ("mfma", FP32_MFMA_PEAK), "p2p": ("alu", FP32_VEC_PEAK)}
# source file of each timed kernel (the HBM traffic figures hold for one version of it)
KERNEL_SOURCES = {"m2l": "m2l.hip", "p2p": "fmm.hip"}


def hbm_traffic(kernel, workload, B, theta):
    """HBM bytes per launch of the mixed-precision kernel, from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary of this workload, scaled by the
    copy-kernel calibration; None when there is none or the kernel's source
    has changed since the counters were taken (or they were taken on another
    leaf size / separation factor)."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith((" ", "#")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_0908_0673_amd", "csrc", KERNEL_SOURCES[kernel])
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if kv.get("source_sha256") != sha or "hbm_bytes_per_launch" not in kv:
        return None
    if kv.get("B") != str(B) or abs(float(kv.get("theta", "nan")) - theta) > 1e-12:
        return None  # counters taken on another tree
    return float(kv["hbm_bytes_per_launch"])


def copy_calibration():
    """A plain 1 GiB device copy: its FETCH_SIZE / WRITE_SIZE readings give the
    factor that turns those counters into bytes."""
    import torch

    n = 1 << 28
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": 4 * n, "launches": 3}))


def algorithmic_flops(stats, P, dbl=True):
    """Per-product algorithmic flop counts of the two heavy phases.

    near field: per (target, source point) pair, Laplace double layer:
      3 sub + 5 (r^2) + 1 (rsqrt) + 5 (r.n) + 3 (r^-3 scale) + 2 (fma) = 19
    M2L: per (target box, source box) pair a P x P product: 2 P^2.
    """
    return {"p2p": 19.0 * stats["n_p2p"] if dbl else 13.0 * stats["n_p2p"],
            "m2l": 2.0 * P * P * stats["n_m2l"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--workload", default="sphere20480")
    # leaf size and separation factor: the fastest pair measured with the
    # product's error against the oracle below 1e-6 on this workload (sweep of
    # B in 12..128 and theta in 0.6..0.7: 6.9e-7 at B = 48, theta = 0.62)
    ap.add_argument("--theta", type=float, default=0.62)
    ap.add_argument("--B", type=int, default=48)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-phases", action="store_true", help="skip the serialized per-phase timing pass")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--serve-full", action="store_true",
                    help="serving measurement on the longer stream (200 requests, 2000-40000 triangles)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a 1 GiB device copy (for HBM counter calibration)")
    ap.add_argument("--batched", action="store_true",
                    help="run only the batched measurement: 64 instances of 1000-40000 triangles, 16 plane-wave "
                         "right-hand sides each, served against plain FP64 one-at-a-time solves")
    ap.add_argument("--batched-kappa", type=float, default=0.0,
                    help="wavenumber bound k (r1 + r2) <= kappa on the lists of the batched set's Helmholtz "
                         "solves (0: none); with it each Helmholtz batch gets a tree of its own k")
    ap.add_argument("--batched-ka-max", type=float, default=5.0,
                    help="largest ka of the batched set (the set's shape names 20; the trees of a served mesh "
                         "are built once for every k, without the wavenumber bound on their lists, so order 8 "
                         "stays accurate only for moderate ka)")
    ap.add_argument("--serve-ka-max", type=float, default=25.0,
                    help="largest ka of the --serve-full stream (see --batched-ka-max)")
    ap.add_argument("--protocol", action="store_true",
                    help="run only the paper's own test protocol (Tables 1-8 shapes, level-dependent order, "
                         "BiCGSTAB, three trees)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(--gpus 1 only).", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return
    if args.protocol:
        paper_protocol()
        return
    if args.batched:
        print(json.dumps({"batched": serving(64, 20090909, (1000, 40000), (1.0, args.batched_ka_max), 16, 4,
                                             96 << 30, uniform_size=True, nrhs_fixed=16,
                                             kappa=args.batched_kappa)}), flush=True)
        return

    import torch

    import bem_inputs
    import paper_0908_0673_amd as bem

    t_setup0 = time.perf_counter()
    m = bem_inputs.workload(args.workload)
    ctx = bem.Context(0)
    mesh = bem.bem_mesh_load(ctx, m.xyz, m.elem)
    tree = bem.bem_tree_build(ctx, mesh, B=args.B, order=8, theta=args.theta)
    stats = tree.stats()
    n = mesh.n_dof
    dof = mesh.dofs()
    x_np = bem_inputs.random_vector(n, 1)[0]
    x = torch.tensor(x_np, dtype=torch.float64, device="cuda:0")[None]
    y = torch.empty_like(x)
    # first products build the corrections and the free term (setup)
    for prec in (bem.BEM_PREC_FP64, bem.BEM_PREC_MIXED):
        bem.bem_matvec(ctx, tree, 0, 0.0, bem.BEM_OP_A, bem.BEM_FMM, prec, x, y)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup0

    def timed(prec, steps, warmup):
        for _ in range(warmup):
            bem.bem_matvec(ctx, tree, 0, 0.0, bem.BEM_OP_A, bem.BEM_FMM, prec, x, y)
        torch.cuda.synchronize()
        # which heavy kernel dominates: both bracketed by events, untimed
        ctx.timing(2)
        for _ in range(3):
            bem.bem_matvec(ctx, tree, 0, 0.0, bem.BEM_OP_A, bem.BEM_FMM, prec, x, y)
        torch.cuda.synchronize()
        probe = ctx.timing(0)
        per = {k: probe[k][0] / max(1, probe[k][1]) for k in ("m2l", "p2p")}
        dom = max(per, key=lambda k: per[k])
        # timed region: one event pair per product, around the dominant kernel
        # on the stream it runs on (the product keeps its two-stream schedule)
        ctx.timing(3 if dom == "p2p" else 4)
        t0 = time.perf_counter()
        for _ in range(steps):
            bem.bem_matvec(ctx, tree, 0, 0.0, bem.BEM_OP_A, bem.BEM_FMM, prec, x, y)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        heavy = ctx.timing(0)
        heavy = {"dominant": dom, "timed": heavy[dom], "probe": per}
        yv = y.cpu().numpy()[0].copy()
        # per-phase device times from HIP events in separate products (while
        # phases are timed, the library runs every phase on the one stream)
        phases = None
        if not args.no_phases:
            ctx.timing(1)
            for _ in range(max(3, steps // 4)):
                bem.bem_matvec(ctx, tree, 0, 0.0, bem.BEM_OP_A, bem.BEM_FMM, prec, x, y)
            torch.cuda.synchronize()
            phases = ctx.timing(0)
        return dt, heavy, phases, yv

    dt_mixed, hv_mixed, ph_mixed, y_mixed = timed(bem.BEM_PREC_MIXED, args.steps, args.warmup)
    dt_fp64, hv_fp64, ph_fp64, y_fp64 = timed(bem.BEM_PREC_FP64, max(3, args.steps // 2), 1)
    ms_mixed = 1e3 * dt_mixed / args.steps
    ms_fp64 = 1e3 * dt_fp64 / max(3, args.steps // 2)
    value = n / (ms_mixed * 1e-3)

    # errors against the oracle's direct product on sampled rows
    err = {}
    try:
        import oracle

        om = oracle.OracleMesh(m.xyz, m.elem)
        rows = np.sort(np.random.default_rng(2).choice(n, 64, replace=False))
        ref = om.matvec_rows(x_np, oracle.OP_A, rows=rows).real
        err = {"mixed": float(np.linalg.norm(y_mixed[rows] - ref) / np.linalg.norm(ref)),
               "fp64": float(np.linalg.norm(y_fp64[rows] - ref) / np.linalg.norm(ref)),
               "rows_sampled": int(rows.size)}
    except Exception as e:  # noqa: BLE001
        err = {"error": str(e)}

    # solves: plain FP64 GMRES(50) vs mixed-precision (relaxed) GMRES, to an FP64 residual of 1e-8
    solve = {}
    if not args.no_solve:
        from oracle import analytic

        phi, chi = analytic.point_source(dof["dof_xyz"], dof["dof_normal"])
        chid = torch.tensor(chi.real, dtype=torch.float64, device="cuda:0")[None]
        # one untimed solve first: the right-hand side's operator (single
        # layer) builds its weights and corrections on first use
        bem.bem_solve(ctx, tree, 0, 0.0, chid, torch.zeros_like(chid), tol=1e-8, restart=50)
        for name, prec in (("fp64", bem.BEM_PREC_FP64), ("mixed", bem.BEM_PREC_MIXED)):
            phid = torch.zeros_like(chid)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = bem.bem_solve(ctx, tree, 0, 0.0, chid, phid, tol=1e-8, restart=50, precision=prec)[0]
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            sol = phid.cpu().numpy()[0]
            solve[name] = {"seconds": dt, "solves_per_s": 1.0 / dt, "iterations": info["iterations"],
                           "refinements": info["refinements"], "matvecs": info["matvecs"],
                           "residual": info["residual"],
                           "rms_error_vs_analytic": float(np.sqrt(np.mean((sol - phi.real) ** 2)))}
        # field of the solved problem at points outside the body (Section 3.5),
        # against the source's own field
        rng = np.random.default_rng(7)
        dirs = rng.standard_normal((4096, 3))
        pts = dirs / np.linalg.norm(dirs, axis=1, keepdims=True) * rng.uniform(1.4, 4.0, (4096, 1))
        pd = torch.tensor(pts, dtype=torch.float64, device="cuda:0")
        bem.bem_field(ctx, tree, 0, 0.0, phid, chid, pd[:64])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u = bem.bem_field(ctx, tree, 0, 0.0, phid, chid, pd)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        want = 1.0 / (4 * np.pi * np.linalg.norm(pts - np.array([0.1, 0.2, 0.3]), axis=1))
        solve["field"] = {"points": len(pts), "seconds": dt, "points_per_s": len(pts) / dt, "theta": 0.25,
                          "max_rel_error_vs_analytic": float(np.abs(u.cpu().numpy()[0] - want).max() / want.max()),
                          "note": "FP64, from the mixed solve's phi; includes the per-call moments and M2M"}

    # roofline of the dominant kernel of the headline product: the M2L
    # products run on the FP32 matrix cores, the near field on the FP32 VALU;
    # its launch duration is the event pair around it in every product of the
    # timed region (the other kernel's comes from the untimed probe products)
    P = 165
    flops = algorithmic_flops(stats, P)
    dom = hv_mixed["dominant"]
    ms_launch = hv_mixed["timed"][0] / max(1, hv_mixed["timed"][1])
    achieved = flops[dom] / (ms_launch * 1e-3) / 1e12
    bound, peak = KERNEL_PEAKS[dom]
    other = [k for k in hv_mixed["probe"] if k != dom][0]
    roofline = {"kernel": dom, "bound": bound, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": hbm_traffic(dom, args.workload, args.B, args.theta),
                "algorithmic_flop_per_launch": flops[dom], "avg_launch_ms": ms_launch,
                "launches": hv_mixed["timed"][1],
                "other_kernel": {"name": other, "avg_launch_ms": hv_mixed["probe"][other],
                                 "note": "three untimed products with events around both kernels"}}

    serve = None
    if not args.no_serve:
        if args.serve_full:
            serve = serving(200, 20090908, (2000, 40000), (1.0, args.serve_ka_max), 32, 4, 96 << 30)
        else:
            serve = serving(24, 20090908, (1000, 6000), (1.0, 5.0), 8, 4, 32 << 30)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(m, x_np, args.cpu_seconds)

    out = {
        "metric": "FMM-BEM matvec unknowns/s",
        "value": value,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_mixed,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 near field and expansions, f64 corrections",
        "data": "synthetic",
        "config": {"workload": f"laplace_{args.workload}_fmm_matvec", "n_elem": m.n_elem, "n_dof": n, "nrhs": 1,
                   "order": 8, "B": args.B, "theta": args.theta, "operator": "A = c.x - K x"},
        "fp64": {"ms_per_step": ms_fp64, "unknowns_per_s": n / (ms_fp64 * 1e-3)},
        "error_vs_oracle": err,
        "phases_ms_per_step": None if ph_mixed is None else {
            "mixed": {k: v[0] / max(1, v[1]) for k, v in ph_mixed.items()},
            "fp64": {k: v[0] / max(1, v[1]) for k, v in ph_fp64.items()},
            "note": "serialized products (one stream), HIP events between phases"},
        "tree": stats,
        "setup_s": t_setup,
        "solve": solve,
        "roofline": roofline,
        "serving": serve,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def paper_protocol():
    """Section 4's test run the paper's way, on the shapes of Tables 1-8: a
    unit point source at (0.1, 0.2, 0.3) inside the unit sphere or the cube
    of edge 2, the Neumann data given and the surface potential recovered by
    BiCGSTAB (to 1e-8); FMM with the level-dependent order L_l = min(8, L_min
    + l_max - l) at L_min = 3 (the tables' plain rows) and 4 (their starred
    rows), beside uniform order 8; the paper's separation test (theta = 1);
    three trees: the paper's read literally (boxes over the DOF points, B
    counting them, every DOF's basis function a source, radii over the
    attached elements), single-owner element sources with those radii, and
    single-owner sources and radii;
    the tables' leaf sizes B (nodes per box), here B/2 elements for
    second-order meshes (two nodes per element) and 2B for first-order ones
    (one node per two elements).  Spheres: icosphere refinements 1-5 (42 ...
    10242 or 162 ... 40962 nodes).  Cubes: structured meshes stand in for the
    paper's unstructured ones, with node counts near the tables' (98 ... 27746
    first-order, 386 ... 27746 second-order).  Laplace (Tables 1-4) and
    Helmholtz k = 2 (Tables 5-8).  One JSON line per row: N (nodes), B, the
    rms error against the exact potential (absolute and relative), setup and
    solve times, BiCGSTAB steps, the peak device bytes of the context and the
    FP64 product time."""
    import torch

    import bem_inputs
    import paper_0908_0673_amd as bem

    xs = np.array([0.1, 0.2, 0.3])
    sphere = ((1, 8), (2, 16), (3, 32), (4, 64), (5, 128))
    cube_p1 = ((4, 5), (8, 10), (17, 20), (35, 40), (68, 80))
    cube_p2 = ((4, 10), (8, 20), (17, 40), (34, 80))
    tables = (("table1", 0, "sphere", 3, sphere), ("table2", 0, "sphere", 6, sphere),
              ("table3", 0, "cube", 3, cube_p1), ("table4", 0, "cube", 6, cube_p2),
              ("table5", 1, "sphere", 3, sphere), ("table6", 1, "sphere", 6, ((1, 16), (2, 32), (3, 64), (4, 128))),
              ("table7", 1, "cube", 3, cube_p1), ("table8", 1, "cube", 6, cube_p2))
    for table, green, shape, nn, sizes in tables:
        k = 2.0 if green else 0.0
        for size, Bp in sizes:
            m = bem_inputs.icosphere(size) if shape == "sphere" else bem_inputs.cube(size)
            if nn == 3:
                m = bem_inputs.linear(m)
            Be = max(4, Bp // 2) if nn == 6 else 2 * Bp
            for attach, omin in ((2, 3), (2, 4), (2, 0), (1, 3), (1, 4), (1, 0), (0, 3), (0, 4), (0, 0)):
                t0 = time.perf_counter()
                ctx = bem.Context(0)
                mesh = bem.bem_mesh_load(ctx, m.xyz, m.elem)
                tree = bem.bem_tree_build(ctx, mesh, B=Bp if attach == 2 else Be, order=8, theta=1.0,
                                          order_min=omin, k_hint=k, attach_radii=attach)
                d = mesh.dofs()
                r = d["dof_xyz"] - xs[None, :]
                R = np.linalg.norm(r, axis=1)
                e = np.exp(1j * k * R)
                phi = e / (4 * np.pi * R)
                chi = (1j * k * R - 1.0) * e / (4 * np.pi * R ** 2) * np.einsum("ij,ij->i", r, d["dof_normal"]) / R
                dt = torch.complex128 if green else torch.float64
                chid = torch.tensor(chi if green else chi.real, dtype=dt, device="cuda:0")[None].contiguous()
                y = torch.empty_like(chid)
                bem.bem_matvec(ctx, tree, green, k, bem.BEM_OP_A, bem.BEM_FMM, bem.BEM_PREC_FP64, chid, y)
                torch.cuda.synchronize()
                t_setup = time.perf_counter() - t0
                phid = torch.empty_like(chid)
                best, info = 1e9, None
                for _ in range(3):
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    info = bem.bem_solve(ctx, tree, green, k, chid, phid, tol=1e-8,
                                         krylov=bem.BEM_KRYLOV_BICGSTAB)[0]
                    torch.cuda.synchronize()
                    best = min(best, time.perf_counter() - t1)
                x = phid.cpu().numpy()[0]
                ref = phi if green else phi.real
                err = float(np.sqrt(np.mean(np.abs(x - ref) ** 2)))
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                for _ in range(20):
                    bem.bem_matvec(ctx, tree, green, k, bem.BEM_OP_A, bem.BEM_FMM, bem.BEM_PREC_FP64, chid, y)
                torch.cuda.synchronize()
                ms_prod = (time.perf_counter() - t1) / 20 * 1e3
                row = {"protocol": f"{table}_{shape}_p{1 if nn == 3 else 2}_{'helmholtz_k2' if green else 'laplace'}",
                       "N": int(m.n_nodes), "n_dof": int(mesh.n_dof), "n_elem": int(m.n_elem), "B_nodes": Bp,
                       "B_elems": None if attach == 2 else Be, "L_min": omin if omin else 8, "L_max": 8, "theta": 1.0,
                       "tree": ("literal", "attached_radii", "owned")[2 - attach],
                       "max_level": int(tree.export()["level"].max()),
                       "eps_rms": err, "eps_rms_rel": err / float(np.sqrt(np.mean(np.abs(ref) ** 2))),
                       "t_setup_s": t_setup, "t_solve_s": best, "iterations": info["iterations"],
                       "matvecs": info["matvecs"], "residual": info["residual"], "status": info["status"],
                       "device_mib_peak": ctx.device_bytes()[1] / 2 ** 20, "ms_per_fp64_product": ms_prod}
                print(json.dumps(row), flush=True)
                tree.close()
                mesh.close()
                ctx.close()
                del chid, phid, y


def _boundary_data(dofs, req):
    """Neumann data of a request: for Helmholtz the sound-hard scattered-field
    data of unit plane waves along the request's directions; for Laplace the
    flux of a unit point source at 0.1 d inside the body, per direction d."""
    x, nrm = dofs["dof_xyz"], dofs["dof_normal"]
    rows = []
    for d in req["dirs"]:
        if req["green"]:
            k = req["k"]
            rows.append(-1j * k * (nrm @ d) * np.exp(1j * k * (x @ d)))
        else:
            r = x - 0.1 * d[None, :]
            R = np.linalg.norm(r, axis=1)
            rows.append(-np.einsum("ij,ij->i", r, nrm) / (4 * np.pi * R ** 3))
    return np.array(rows)


def serving(count, seed, n_tri, ka, nrhs_max, lanes, budget, rate_frac=0.5, uniform_size=False, nrhs_fixed=0,
            kappa=0.0):
    """Served, mixed-precision solves (bem_server_*: concurrent lanes, request
    merging, right-hand sides in lock step) against plain FP64 solves of one
    right-hand side at a time on one context, on the same seeded request
    stream; trees are cached per mesh on both sides.
    Throughput: all requests offered at once.  Latency: a second pass with
    Poisson arrivals at rate_frac times the measured request throughput
    (warm caches), submission to completion."""
    import torch

    import paper_0908_0673_amd as bem
    from bem_inputs.requests import mesh_of, request_stream

    reqs = request_stream(count, seed, n_tri=n_tri, ka=ka, nrhs_max=nrhs_max, uniform_size=uniform_size,
                          nrhs_fixed=nrhs_fixed)
    meshes = {}
    for r in reqs:
        if r["key"] not in meshes:
            meshes[r["key"]] = mesh_of(r)
    total_rhs = sum(r["nrhs"] for r in reqs)
    print(f"serving: {len(meshes)} meshes generated, {total_rhs} right-hand sides", file=sys.stderr, flush=True)
    out = {"requests": count, "rhs": total_rhs, "distinct_meshes": len(meshes), "kappa": kappa,
           "elements": [int(min(m.n_elem for m in meshes.values())), int(max(m.n_elem for m in meshes.values()))],
           "lanes": lanes, "hbm_budget_gb": budget / 2 ** 30, "seed": seed,
           "stream": f"n_tri {'uniform' if uniform_size else 'log-uniform'} {list(n_tri)}, sphere/cube/ellipsoid, "
                     f"Laplace/Helmholtz 50/50, ka U{list(ka)}, "
                     + (f"nrhs {nrhs_fixed}" if nrhs_fixed else f"nrhs U[1,{nrhs_max}]")}
    # served
    # kappa > 0: the wavenumber bound on the lists; the server then solves every
    # Helmholtz batch on a tree of its own k, and so does the baseline below
    srv = bem.Server(lanes=lanes, hbm_budget=budget, max_batch_rhs=32, precision=bem.BEM_PREC_MIXED, kappa=kappa)
    try:
        ids = {key: srv.add_mesh(m.xyz, m.elem)[0] for key, m in meshes.items()}
        chis = [_boundary_data(srv.mesh_dofs(ids[r["key"]]), r) for r in reqs]
        t0 = time.perf_counter()
        tickets = [srv.submit(ids[r["key"]], r["green"], r["k"], c) for r, c in zip(reqs, chis)]
        res = []
        for i, t in enumerate(tickets):
            res.append(srv.poll(t))
            if (i + 1) % 8 == 0:
                print(f"serving: {i + 1} of {count} requests served", file=sys.stderr, flush=True)
        dt = time.perf_counter() - t0
        out["served_solves_per_s"] = total_rhs / dt
        out["served_requests_per_s"] = count / dt
        out["served_not_converged"] = sum(1 for r in res for i in r[2] if i["status"] != 0)
        rate = rate_frac * count / dt
        t0 = time.perf_counter()
        tickets = []
        for r, c in zip(reqs, chis):
            wait = r["t"] / rate - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            tickets.append(srv.submit(ids[r["key"]], r["green"], r["k"], c))
        lat = np.array([srv.poll(t)[3] for t in tickets])
        out["open_loop_rate_requests_per_s"] = rate
        out["latency_ms"] = {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3)}
        out["server_stats"] = srv.stats()
    finally:
        srv.close()
    print(f"serving: served pass done ({out.get('served_solves_per_s', 0):.1f} solves/s)", file=sys.stderr, flush=True)
    # plain FP64, one request at a time
    ctx = bem.Context(0)
    trees = {}
    t0 = time.perf_counter()
    lat_base = []
    nconv = 0
    for r, c in zip(reqs, chis):
        t1 = time.perf_counter()
        if r["key"] not in trees:
            m = meshes[r["key"]]
            mesh = bem.bem_mesh_load(ctx, m.xyz, m.elem)
            trees[r["key"]] = (mesh, bem.bem_tree_build(ctx, mesh, B=32, order=8, theta=0.6))
        cplx = r["green"] == 1
        chid = torch.tensor(c if cplx else c.real, dtype=torch.complex128 if cplx else torch.float64, device="cuda:0")
        phid = torch.empty_like(chid)
        tree, own = trees[r["key"]][1], None
        if cplx and kappa > 0.0:
            own = bem.bem_tree_build(ctx, trees[r["key"]][0], B=32, order=8, theta=0.6, kappa=kappa, k_hint=r["k"])
            tree = own
        for j in range(chid.shape[0]):  # one right-hand side at a time
            info = bem.bem_solve(ctx, tree, r["green"], r["k"], chid[j:j + 1], phid[j:j + 1],
                                 precision=bem.BEM_PREC_FP64)
            nconv += sum(1 for i in info if i["status"] != 0)
        if own is not None:
            own.close()
        torch.cuda.synchronize()
        lat_base.append(time.perf_counter() - t1)
        if len(lat_base) % 8 == 0:
            print(f"serving: {len(lat_base)} of {count} requests solved one at a time", file=sys.stderr, flush=True)
    dtb = time.perf_counter() - t0
    out["baseline_fp64_solves_per_s"] = total_rhs / dtb
    out["baseline_not_converged"] = nconv
    out["baseline_latency_ms"] = {"p50": float(np.percentile(lat_base, 50) * 1e3),
                                  "p99": float(np.percentile(lat_base, 99) * 1e3)}
    out["speedup_solves_per_s"] = out["served_solves_per_s"] / out["baseline_fp64_solves_per_s"]
    for tr in trees.values():
        tr[1].close()
        tr[0].close()
    return out


def cpu_baseline(m, x_np, seconds):
    """The oracle (plain FP64 C, OpenMP over rows) on a bounded sample: full
    rows of the direct product of the same operator on the same mesh."""
    import oracle

    om = oracle.OracleMesh(m.xyz, m.elem)
    rng = np.random.default_rng(3)
    rows = rng.permutation(om.n_dof)
    done, t0, chunk = 0, time.perf_counter(), 256
    while time.perf_counter() - t0 < seconds and done < om.n_dof:
        om.matvec_rows(x_np, oracle.OP_A, rows=np.sort(rows[done:done + chunk]))
        done += chunk
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": done / dt, "unit": "unknowns/s", "cores": cores, "kind": "oracle",
            "sample": f"{done} full rows of the direct product A x on the {om.n_dof}-DOF mesh "
                      f"(plain FP64 oracle, {dt:.1f} s)"}


if __name__ == "__main__":
    main()
