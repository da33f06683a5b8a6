"""Benchmark: fast-multipole BEM matrix-vector products and solves on one MI355X.

Workloads (the fast product of the system operator A x = c.x - K x, order-8
expansions, input already in device memory; each tree's leaf size, separation
factor and wavenumber bound are the cheapest of a sweep whose largest error
over all rows stays below 1e-6 against the FP64 direct product):

  c2_sphere  Laplace, unit sphere of 20480 curved 6-node triangles (40962
             DOFs), B = 48, theta = 0.5
  c2_cube    Laplace, cube [-1, 1]^3 of 24300 triangles with sharp edges
             (49686 DOFs), B = 48, theta = 0.55
  c3         Helmholtz ka = 10, geodesic sphere of 30420 triangles (60842
             complex DOFs), B = 64, theta = 0.5, k (r1 + r2) <= 2.2

A step is one mixed-precision product (single-precision near field and
expansions, double-precision corrections, free term and combination) on each
of the two meshes of the C2 configuration, the one the metric is quoted on;
the headline value is their unknowns per second.  C3, the plain FP64
products, GMRES(50) solves to a 1e-8 FP64 residual (plain FP64 against mixed
precision), errors against the oracle (sampled rows, 2-norm and largest row),
per-phase device times, every workload's dominant-kernel roofline, the
serving measurement and the CPU oracle are reported beside it.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-serve] [--no-c3]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP32_VEC_PEAK = 157.3  # TFLOP/s, MI355X vector FP32 (256 CUs x 2.4 GHz; counts packed FP32)
FP32_VEC_UNPACKED = 78.6  # TFLOP/s: the same without packed FP32, which this build does not emit
FP32_MFMA_PEAK = 157.3  # TFLOP/s, MI355X dense FP32 matrix
FP64_VEC_PEAK = 78.6
FP16_MFMA_PEAK = 2500.0  # TFLOP/s: dense fp16 matrix peak (the split M2L's instruction)
KERNEL_PEAKS = {"m2l": ("mfma", FP32_MFMA_PEAK), "p2p": ("alu", FP32_VEC_PEAK)}
# leaf sizes of the served trees: Laplace, and Helmholtz per wavenumber bucket
# (the C3 sweep: B = 64 is 5.6 times faster than B = 32 at ka = 10)
SERVE_B, SERVE_B_HELMHOLTZ = 48, 64
# source file of each timed kernel (the HBM traffic figures hold for one version of it)
KERNEL_SOURCES = {"m2l": "m2l.hip", "p2p": "fmm.hip"}

# name -> (mesh, Green's function, k, B, theta, kappa)
WORKLOADS = {
    "c2_sphere": ("sphere20480", 0, 0.0, 48, 0.5, 0.0),
    "c2_cube": ("cube24300", 0, 0.0, 48, 0.55, 0.0),
    "c3": ("geodesic30420", 1, 10.0, 64, 0.5, 2.2),
}
HEADLINE = ("c2_sphere", "c2_cube")


def code_sha256(path):
    """Hash of a source file's code: comments, blank lines and the
    indentation of lines removed (a change of comments only keeps it)."""
    import re

    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = [re.sub(r"//.*$", "", ln).strip() for ln in text.splitlines()]
    return hashlib.sha256("\n".join(ln for ln in lines if ln).encode()).hexdigest()


def hbm_traffic(kernel, mesh, B, theta, kappa):
    """HBM bytes per launch of the mixed-precision kernel on this tree, from
    the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary, scaled by the
    copy-kernel calibration; None when there is none or the kernel's source
    has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{mesh}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith((" ", "#")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_0908_0673_amd", "csrc", KERNEL_SOURCES[kernel])
    if kv.get("code_sha256") != code_sha256(src) or "hbm_bytes_per_launch" not in kv:
        return None
    try:
        same = (int(kv.get("B", -1)) == B and abs(float(kv.get("theta", "nan")) - theta) < 1e-12
                and abs(float(kv.get("kappa", "0")) - kappa) < 1e-12)
    except ValueError:
        same = False
    return float(kv["hbm_bytes_per_launch"]) if same else None


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


def algorithmic_flops(stats, P, helm):
    """Per-product algorithmic flop counts of the two heavy phases (operator A,
    double layer).

    near field, per (target, source point) pair, as the mixed-precision kernel
    evaluates it (a transcendental instruction counted as one):
      Laplace:   3 (difference) + 5 (r^2) + 1 (1/r) + 5 (r.n) + 3 (r^-3) + 2 (accumulate) = 19
      Helmholtz: 3 + 5 + 1 + 2 (k r) + 4 (turns, fraction, sin, cos) + 5 (r.n) + 3 (r.n / r^3)
                 + 4 (cos + kr sin, sin - kr cos) + 2 (scaling) + 8 (complex strength and
                 accumulate) = 37
    M2L: per (target box, source box) pair a P x P product, 2 P^2 real, 8 P^2 complex.
    """
    return {"p2p": (37.0 if helm else 19.0) * stats["n_p2p"],
            "m2l": (8.0 if helm else 2.0) * P * P * stats["n_m2l"]}


class Workload:
    """One tree of one named workload on the shared context, with its input."""

    def __init__(self, ctx, name):
        import torch

        import bem_inputs
        import paper_0908_0673_amd as bem

        self.bem, self.ctx, self.name = bem, ctx, name
        self.mesh_name, self.green, self.k, self.B, self.theta, self.kappa = WORKLOADS[name]
        t0 = time.perf_counter()
        self.m = bem_inputs.workload(self.mesh_name)
        self.mesh = bem.bem_mesh_load(ctx, self.m.xyz, self.m.elem)
        self.tree = bem.bem_tree_build(ctx, self.mesh, B=self.B, order=8, theta=self.theta, kappa=self.kappa,
                                       k_hint=self.k)
        self.n = self.mesh.n_dof
        self.cplx = self.green == 1
        self.x_np = bem_inputs.random_vector(self.n, 1, complex_=self.cplx)[0]
        dt = torch.complex128 if self.cplx else torch.float64
        self.x = torch.tensor(self.x_np if self.cplx else self.x_np.real, dtype=dt, device="cuda:0")[None].contiguous()
        self.y = torch.empty_like(self.x)
        for prec in (0, 1):  # the first products build corrections, free term, plans (setup)
            self.product(prec)
        torch.cuda.synchronize()
        self.setup_s = time.perf_counter() - t0
        self.stats = self.tree.stats(self.green, self.k)

    def product(self, prec, op=2):
        self.bem.bem_matvec(self.ctx, self.tree, self.green, self.k, op, self.bem.BEM_FMM, prec, self.x, self.y)

    def config(self):
        return {"workload": f"{'helmholtz_ka10' if self.cplx else 'laplace'}_{self.mesh_name}_fmm_matvec",
                "n_elem": self.m.n_elem, "n_dof": self.n, "value_type": "complex" if self.cplx else "real",
                "nrhs": 1, "order": 8, "B": self.B, "theta": self.theta, "kappa": self.kappa or None,
                "k": self.k or None, "operator": "A = c.x - K x"}


def probe_dominant(ctx, wls, prec):
    """Average launch time of the two heavy kernels over three untimed
    products of each workload (events around both, the usual scheduling)."""
    import torch

    out = {}
    for w in wls:
        ctx.timing(2)
        for _ in range(3):
            w.product(prec)
        torch.cuda.synchronize()
        ph = ctx.timing(0)
        out[w.name] = {k: ph[k][0] / max(1, ph[k][1]) for k in ("m2l", "p2p")}
    return out


def timed_products(ctx, wls, prec, steps, warmup, dom):
    """steps x (one product of every workload in wls), with one event pair per
    product around the kernel `dom` (on its stream); returns wall ms per step
    and the event-timed (ms, launches) of that kernel."""
    import torch

    for _ in range(warmup):
        for w in wls:
            w.product(prec)
    torch.cuda.synchronize()
    ctx.timing(3 if dom == "p2p" else 4)
    t0 = time.perf_counter()
    for _ in range(steps):
        for w in wls:
            w.product(prec)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ph = ctx.timing(0)
    return 1e3 * dt / steps, ph[dom]


def phase_times(ctx, w, prec, reps):
    import torch

    ctx.timing(1)
    for _ in range(reps):
        w.product(prec)
    torch.cuda.synchronize()
    ph = ctx.timing(0)
    return {k: v[0] / max(1, v[1]) for k, v in ph.items()}


def oracle_errors(w, yv, rows_n=64):
    """Sampled rows of the oracle's direct product against y: 2-norm and
    largest-row relative errors."""
    import oracle

    om = oracle.OracleMesh(w.m.xyz, w.m.elem)
    rows = np.sort(np.random.default_rng(2).choice(w.n, rows_n, replace=False))
    ref = om.matvec_rows(w.x_np, oracle.OP_A, green=w.green, k=w.k, rows=rows)
    if not w.cplx:
        ref = ref.real
    out = {}
    for name, y in yv.items():
        d = np.abs(y[rows] - ref)
        out[name] = {"rel_2norm": float(np.linalg.norm(d) / np.linalg.norm(ref)),
                     "rel_max_row": float(d.max() / np.abs(ref).max())}
    out["rows_sampled"] = int(rows.size)
    return out


def roofline(dom, flops, ms_launch, launches, traffic):
    bound, peak = KERNEL_PEAKS[dom]
    achieved = flops / (ms_launch * 1e-3) / 1e12
    r = {"kernel": dom, "bound": bound, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
         "frac": achieved / peak, "traffic": traffic, "algorithmic_flop_per_launch": flops,
         "avg_launch_ms": ms_launch, "launches": launches}
    if dom == "p2p":  # the attainable VALU peak of a build without packed FP32
        r["peak_unpacked"] = FP32_VEC_UNPACKED
        r["frac_unpacked"] = achieved / FP32_VEC_UNPACKED
    if dom == "m2l":
        # the mixed-precision products run on the fp16 matrix instruction with
        # two-term operand splits: three products per FP32-equivalent one, on
        # a 176 x 192 padded tile per P x P block
        ex = achieved * 3 * (176 * 192) / (165 * 165)
        r["fp16_executed_tflops"] = ex
        r["fp16_peak"] = FP16_MFMA_PEAK
        r["fp16_frac"] = ex / FP16_MFMA_PEAK
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the Helmholtz ka = 10 workload")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-fmm", action="store_true", help="skip timing the oracle's fast product")
    ap.add_argument("--no-phases", action="store_true", help="skip the serialized per-phase timing pass")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a 1 GiB device copy (for HBM counter calibration)")
    ap.add_argument("--batched", action="store_true",
                    help="run only the batched measurement: 64 instances of 1000-40000 triangles, 16 plane-wave "
                         "right-hand sides each, served against plain FP64 one-at-a-time solves")
    ap.add_argument("--batched-kappa", type=float, default=2.2,
                    help="wavenumber bound k (r1 + r2) <= kappa on the lists of the Helmholtz trees")
    ap.add_argument("--batched-ka-max", type=float, default=20.0, help="largest ka of the batched set")
    ap.add_argument("--serve-c5", action="store_true",
                    help="run only the serving stream of the C5 shape: Poisson arrivals, 2000-80000 triangles "
                         "log-uniform, Laplace/Helmholtz 50/50, ka 1-25, 1-32 right-hand sides, rate swept over "
                         "fractions of the saturation rate")
    ap.add_argument("--c5-count", type=int, default=1000, help="counted requests of --serve-c5")
    ap.add_argument("--c5-warmup", type=int, default=50, help="warm-up requests of --serve-c5")
    ap.add_argument("--c5-fracs", default="0.25,0.5,0.8,1.0", help="rates of --serve-c5 as fractions of saturation")
    ap.add_argument("--c5-baseline", type=int, default=0,
                    help="plain FP64 service times on the first this many counted requests (0: all)")
    ap.add_argument("--lanes", type=int, default=4, help="serving lanes")
    ap.add_argument("--max-seconds", type=float, default=60.0, help="time budget per served batch")
    ap.add_argument("--protocol", action="store_true",
                    help="run only the paper's own test protocol (Tables 1-8 shapes, level-dependent order, "
                         "BiCGSTAB, three trees)")
    ap.add_argument("--only", default="", help="comma-separated workloads to set up (profiling runs)")
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
    if args.batched:  # C4: 64 instances, 1000-40000 triangles, ka 1-20, 16 plane waves each, all at once
        print(json.dumps({"batched": serving(64, 20090909, (1000, 40000), (1.0, args.batched_ka_max), 16,
                                             args.lanes, 96 << 30, rate_fracs=(), uniform_size=True, nrhs_fixed=16,
                                             kappa=args.batched_kappa, max_seconds=args.max_seconds,
                                             label="batched")}), flush=True)
        return
    if args.serve_c5:  # C5: Poisson stream, 2000-80000 triangles, ka 1-25, 1-32 right-hand sides
        fr = tuple(float(f) for f in args.c5_fracs.split(","))
        print(json.dumps({"serving_c5": serving(args.c5_count, 20090910, (2000, 80000), (1.0, 25.0), 32,
                                                args.lanes, 96 << 30, rate_fracs=fr, kappa=2.2,
                                                max_seconds=args.max_seconds, warmup=args.c5_warmup,
                                                baseline_count=args.c5_baseline or None, label="c5")}),
              flush=True)
        return

    import torch

    import paper_0908_0673_amd as bem

    ctx = bem.Context(0)
    names = [n for n in WORKLOADS if not (args.no_c3 and n == "c3")]
    if args.only:
        names = [n for n in names if n in args.only.split(",")]
    wls = {}
    for n in names:
        wls[n] = Workload(ctx, n)
        print(f"bench: {n} set up ({wls[n].setup_s:.2f} s)", file=sys.stderr, flush=True)
    head = [wls[n] for n in HEADLINE if n in wls]

    # every workload on its own: dominant kernel, event-timed products, errors
    per = {}
    P = 165
    for n, w in wls.items():
        probe = probe_dominant(ctx, [w], bem.BEM_PREC_MIXED)[n]
        dom = max(probe, key=lambda k: probe[k])
        steps_w = max(5, args.steps // (5 if w.cplx else 1))
        ms = {}
        ys = {}
        dom_t = None
        for prec, pname in ((bem.BEM_PREC_MIXED, "mixed"), (bem.BEM_PREC_FP64, "fp64")):
            ms_step, kt = timed_products(ctx, [w], prec, steps_w if prec else max(3, steps_w // 2), 3, dom)
            ms[pname] = ms_step
            if prec == bem.BEM_PREC_MIXED:
                dom_t = kt
            w.product(prec)
            torch.cuda.synchronize()
            ys[pname] = w.y.cpu().numpy()[0].copy()
        fl = algorithmic_flops(w.stats, P, w.cplx)
        ms_launch = dom_t[0] / max(1, dom_t[1])
        per[n] = {"config": w.config(),
                  "ms_per_product": ms,
                  "unknowns_per_s": {k: w.n / (v * 1e-3) for k, v in ms.items()},
                  "error_vs_oracle": oracle_errors(w, ys),
                  "roofline": roofline(dom, fl[dom], ms_launch, dom_t[1],
                                       hbm_traffic(dom, w.mesh_name, w.B, w.theta, w.kappa)),
                  "other_kernel_ms": {k: v for k, v in probe.items() if k != dom},
                  "tree": w.stats, "setup_s": w.setup_s}
        if not args.no_phases:
            per[n]["phases_ms"] = {pname: phase_times(ctx, w, prec, 5)
                                   for prec, pname in ((bem.BEM_PREC_MIXED, "mixed"), (bem.BEM_PREC_FP64, "fp64"))}
        print(f"bench: {n} measured ({ms['mixed']:.3f} ms mixed, {ms['fp64']:.3f} ms fp64)", file=sys.stderr,
              flush=True)

    # the headline step: one mixed product on each C2 mesh; events around the
    # kernel that dominates the step
    out = {"metric": "FMM-BEM matvec unknowns/s", "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 near field and expansions, f64 corrections", "data": "synthetic"}
    if head:
        tot = {k: sum(per[w.name]["other_kernel_ms"].get(k, 0.0) + (
            per[w.name]["roofline"]["avg_launch_ms"] if per[w.name]["roofline"]["kernel"] == k else 0.0)
            for w in head) for k in ("m2l", "p2p")}
        dom = max(tot, key=lambda k: tot[k])
        ms_step, kt = timed_products(ctx, head, bem.BEM_PREC_MIXED, args.steps, args.warmup, dom)
        n_head = sum(w.n for w in head)
        flops = sum(algorithmic_flops(w.stats, P, w.cplx)[dom] for w in head) / len(head)
        traffic = [hbm_traffic(dom, w.mesh_name, w.B, w.theta, w.kappa) for w in head]
        out.update({
            "value": n_head / (ms_step * 1e-3), "ms_per_step": ms_step,
            "config": {"workload": "laplace_c2_sphere20480_and_cube24300_fmm_matvec",
                       "meshes": [w.config() for w in head], "n_dof_per_step": n_head,
                       "step": "one mixed-precision product of A on each mesh"},
            "roofline": roofline(dom, flops, kt[0] / max(1, kt[1]), kt[1],
                                 None if None in traffic else sum(traffic) / len(traffic)),
        })
        out["roofline"]["note"] = ("averages over the step's launches on both meshes (flops and traffic per "
                                   "launch averaged the same way)")
    out["workloads"] = per

    # solves: plain FP64 GMRES(50) vs mixed-precision (relaxed) GMRES, to an FP64 residual of 1e-8
    if not args.no_solve:
        out["solve"] = solves(bem, ctx, wls)

    if not args.no_serve:  # a bounded slice of the C5 stream's shape
        out["serving"] = serving(32, 20090908, (2000, 20000), (1.0, 25.0), 8, 4, 32 << 30, rate_fracs=(0.5,),
                                 kappa=2.2, max_seconds=10.0, warmup=4, label="serving")
        out["serving"]["slice"] = ("the C5 shape bounded for the default run: 32 requests after 4 warm-up, "
                                   "2000-20000 triangles, 1-8 right-hand sides, 32 GiB budget")

    if not args.no_cpu and "c2_sphere" in wls:
        w = wls["c2_sphere"]
        out["cpu_baseline"] = cpu_baseline(w.m, w.x_np, args.cpu_seconds, fmm=not args.no_cpu_fmm, B=w.B,
                                           theta=w.theta)
    print(json.dumps(out), flush=True)


def solves(bem, ctx, wls):
    """Plain FP64 against mixed-precision GMRES(50) to an FP64 residual of
    1e-8: point-source data on the C2 meshes, the rigid-sphere plane wave on
    C3 (against the series solution)."""
    import torch

    from oracle import analytic

    res = {}
    for n, w in wls.items():
        d = w.mesh.dofs()
        if w.cplx:
            inc, chi = analytic.plane_wave(d["dof_xyz"], d["dof_normal"], w.k)
            ref = analytic.rigid_sphere_total(w.k, d["dof_xyz"][:, 2] / np.linalg.norm(d["dof_xyz"], axis=1))
            chid = torch.tensor(chi, dtype=torch.complex128, device="cuda:0")[None].contiguous()
        else:
            phi, chi = analytic.point_source(d["dof_xyz"], d["dof_normal"])
            chid = torch.tensor(chi.real, dtype=torch.float64, device="cuda:0")[None].contiguous()
        # one untimed solve first: the right-hand side's operator builds its tables on first use
        bem.bem_solve(ctx, w.tree, w.green, w.k, chid, torch.zeros_like(chid), tol=1e-8, restart=50)
        r = {}
        for name, prec in (("fp64", bem.BEM_PREC_FP64), ("mixed", bem.BEM_PREC_MIXED)):
            phid = torch.zeros_like(chid)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = bem.bem_solve(ctx, w.tree, w.green, w.k, chid, phid, tol=1e-8, restart=50, precision=prec)[0]
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            sol = phid.cpu().numpy()[0]
            e = {"seconds": dt, "solves_per_s": 1.0 / dt, "iterations": info["iterations"],
                 "restarts": info["restarts"], "matvecs": info["matvecs"], "residual": info["residual"],
                 "status": info["status"]}
            if w.cplx:
                tot = sol + inc
                e["rms_rel_error_vs_series"] = float(np.linalg.norm(tot - ref) / np.linalg.norm(ref))
            else:
                e["rms_error_vs_analytic"] = float(np.sqrt(np.mean((sol - phi.real) ** 2)))
            r[name] = e
        res[n] = r
        print(f"bench: {n} solves done", file=sys.stderr, flush=True)
    if "c2_sphere" in wls:  # field of the solved problem at points outside the body (Section 3.5)
        w = wls["c2_sphere"]
        d = w.mesh.dofs()
        phi_a, chi = analytic.point_source(d["dof_xyz"], d["dof_normal"])
        chid = torch.tensor(chi.real, dtype=torch.float64, device="cuda:0")[None].contiguous()
        phid = torch.zeros_like(chid)
        bem.bem_solve(ctx, w.tree, 0, 0.0, chid, phid, tol=1e-8, precision=bem.BEM_PREC_MIXED)
        rng = np.random.default_rng(7)
        dirs = rng.standard_normal((4096, 3))
        pts = dirs / np.linalg.norm(dirs, axis=1, keepdims=True) * rng.uniform(1.4, 4.0, (4096, 1))
        pd = torch.tensor(pts, dtype=torch.float64, device="cuda:0")
        bem.bem_field(ctx, w.tree, 0, 0.0, phid, chid, pd[:64])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u = bem.bem_field(ctx, w.tree, 0, 0.0, phid, chid, pd)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        want = 1.0 / (4 * np.pi * np.linalg.norm(pts - np.array([0.1, 0.2, 0.3]), axis=1))
        res["field_c2_sphere"] = {
            "points": len(pts), "seconds": dt, "points_per_s": len(pts) / dt, "theta": 0.25,
            "max_rel_error_vs_analytic": float(np.abs(u.cpu().numpy()[0] - want).max() / want.max()),
            "note": "FP64, from the mixed solve's phi; includes the per-call moments and M2M"}
    return res


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


def _bucket_top(k):
    """Top of the server's wavenumber bucket of k: 2^(ceil(4 log2 k) / 4)."""
    return float(2.0 ** (np.ceil(4.0 * np.log2(k) - 1e-12) / 4.0))


_JN_ZEROS = None


def _jn_zero_distance(ka):
    """Distance of ka to the nearest zero of a spherical Bessel function j_n
    (n <= 60): the exterior Neumann equation without a Burton-Miller
    correction is singular there on the unit sphere."""
    global _JN_ZEROS
    if _JN_ZEROS is None:
        from scipy.optimize import brentq
        from scipy.special import spherical_jn

        zs = []
        x = np.linspace(0.05, 45.0, 45001)
        for n in range(61):
            v = spherical_jn(n, x)
            for i in np.nonzero(np.sign(v[:-1]) * np.sign(v[1:]) < 0)[0]:
                zs.append(brentq(lambda t: spherical_jn(n, t), x[i], x[i + 1]))
        _JN_ZEROS = np.sort(np.array(zs))
    return float(np.abs(_JN_ZEROS - ka).min())


def serving(count, seed, n_tri, ka, nrhs_max, lanes, budget, rate_fracs=(0.5,), uniform_size=False, nrhs_fixed=0,
            kappa=2.2, max_iters=1000, max_seconds=60.0, warmup=0, baseline_count=None, label="serving"):
    """Served, mixed-precision solves (bem_server_*: concurrent lanes, request
    merging, right-hand sides in lock step, trees kept per mesh and
    wavenumber bucket under the device-memory budget) against plain FP64
    solves of one request and one right-hand side at a time on one context,
    on the same seeded request stream and the same trees.

    The first `warmup` requests are served and not counted.  Throughput: the
    next `count` requests offered at once (the saturation rate).  Latency:
    for each fraction f of rate_fracs, the same requests again as a Poisson
    stream at f times the saturation rate (open loop, submission to
    completion).  Baseline: the FP64 service time of every counted request
    (or of the first baseline_count), its throughput, and its latency under
    the same arrivals as a single first-come-first-served server (completion
    = max(arrival, previous completion) + service time), so the two latency
    figures are measured against the same arrival process.  Every solve has
    the step budget max_iters per right-hand side and the time budget
    max_seconds per batch (non-converged counts reported on both sides), and
    for Helmholtz requests on spheres the distance of ka to the nearest zero
    of a spherical Bessel function is reported (irregular frequencies)."""
    import torch

    import paper_0908_0673_amd as bem
    from bem_inputs.requests import mesh_of, request_stream

    reqs_all = request_stream(count + warmup, seed, n_tri=n_tri, ka=ka, nrhs_max=nrhs_max, uniform_size=uniform_size,
                              nrhs_fixed=nrhs_fixed)
    t0 = time.perf_counter()
    meshes = {}
    for r in reqs_all:
        if r["key"] not in meshes:
            meshes[r["key"]] = mesh_of(r)
    warm, reqs = reqs_all[:warmup], reqs_all[warmup:]
    total_rhs = sum(r["nrhs"] for r in reqs)
    print(f"{label}: {len(meshes)} meshes generated in {time.perf_counter() - t0:.1f} s, {len(reqs)} requests "
          f"({total_rhs} right-hand sides) after {warmup} warm-up", file=sys.stderr, flush=True)
    sizes = [meshes[r["key"]].n_elem for r in reqs]
    out = {"requests": count, "warmup_requests": warmup, "rhs": total_rhs, "distinct_meshes": len(meshes),
           "kappa": kappa, "elements": [int(min(sizes)), int(max(sizes))], "mean_elements": float(np.mean(sizes)),
           "lanes": lanes, "hbm_budget_gb": budget / 2 ** 30, "seed": seed, "max_iters": max_iters,
           "max_seconds_per_batch": max_seconds,
           "stream": f"n_tri {'uniform' if uniform_size else 'log-uniform'} {list(n_tri)}, sphere/cube/ellipsoid, "
                     f"Laplace/Helmholtz 50/50, ka U{list(ka)} (k = ka / circumradius), "
                     + (f"nrhs {nrhs_fixed}" if nrhs_fixed else f"nrhs U[1,{nrhs_max}]")}
    sph = [r for r in reqs if r["green"] and r["shape"] == "sphere"]
    if sph:
        d = np.array([_jn_zero_distance(r["ka"]) for r in sph])
        out["sphere_helmholtz_jn_zero_distance"] = {"requests": len(sph), "min": float(d.min()),
                                                    "median": float(np.median(d)),
                                                    "below_0.05": int((d < 0.05).sum())}

    def summary(results):
        infos = [i for r in results for i in r[2]]
        it = np.array([i["iterations"] for i in infos]) if infos else np.zeros(1)
        return {"not_converged": sum(1 for i in infos if i["status"] != 0),
                "failed_requests": sum(1 for r in results if r[0] not in (0, bem.BEM_ENOCONV)),
                "iterations": {"median": float(np.median(it)), "max": int(it.max()), "mean": float(it.mean())}}

    srv = bem.Server(lanes=lanes, hbm_budget=budget, max_batch_rhs=32, precision=bem.BEM_PREC_MIXED, kappa=kappa,
                     max_iters=max_iters, max_seconds=max_seconds, B=SERVE_B, helmholtz_B=SERVE_B_HELMHOLTZ)
    try:
        ids = {key: srv.add_mesh(m.xyz, m.elem)[0] for key, m in meshes.items()}
        dofs = {key: srv.mesh_dofs(i) for key, i in ids.items()}

        def submit(r):
            return srv.submit(ids[r["key"]], r["green"], r["k"], _boundary_data(dofs[r["key"]], r))

        if warm:
            for i, t in enumerate([submit(r) for r in warm]):
                srv.poll(t)
                print(f"{label}: warm-up {i + 1} of {len(warm)} served", file=sys.stderr, flush=True)
            print(f"{label}: warm-up served", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        tickets = [submit(r) for r in reqs]
        res = []
        for i, t in enumerate(tickets):
            rc, phi, info, lat = srv.poll(t)
            res.append((rc, None, info, lat))
            r = reqs[i]
            print(f"{label}: {i + 1} of {len(reqs)} requests served at {time.perf_counter() - t0:.1f} s "
                  f"({r['n_tri']} tri, green {r['green']}, ka {r['ka']:.2f}, nrhs {r['nrhs']}, rc {rc})",
                  file=sys.stderr, flush=True)
        dt = time.perf_counter() - t0
        sat = len(reqs) / dt
        out["served_solves_per_s"] = total_rhs / dt
        out["served_requests_per_s"] = sat
        out["served"] = summary(res)
        print(f"{label}: partial {json.dumps(out)}", file=sys.stderr, flush=True)
        out["open_loop"] = []
        arrivals = np.array([r["t"] for r in reqs])
        arrivals = arrivals - arrivals[0]
        for f in rate_fracs:
            rate = f * sat
            t0 = time.perf_counter()
            tickets = []
            for r, a_ in zip(reqs, arrivals):
                wait = a_ / rate - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
                tickets.append(submit(r))
                print(f"{label}: open loop at {f}: {len(tickets)} of {len(reqs)} submitted", file=sys.stderr,
                      flush=True)
            lat = []
            for i, t in enumerate(tickets):
                lat.append(srv.poll(t)[3])
                print(f"{label}: open loop at {f}: {i + 1} of {len(tickets)} done", file=sys.stderr, flush=True)
            lat = np.array(lat)
            out["open_loop"].append({"rate_fraction_of_saturation": f, "rate_requests_per_s": rate,
                                     "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                                                    "p99": float(np.percentile(lat, 99) * 1e3)}})
            print(f"{label}: open loop at {f} x saturation done: {json.dumps(out['open_loop'][-1])}", file=sys.stderr,
                  flush=True)
        out["server_stats"] = srv.stats()
    finally:
        srv.close()
    print(f"{label}: served ({out.get('served_solves_per_s', 0):.1f} solves/s)", file=sys.stderr, flush=True)
    # plain FP64, one request at a time, one right-hand side at a time, on the
    # trees the server uses (per mesh and, with the wavenumber bound, per
    # wavenumber bucket), cached on first use (least recently used dropped
    # beyond the budget's worth of meshes)
    ctx = bem.Context(0)
    meshes_dev, trees = {}, {}
    base = reqs if baseline_count is None else reqs[:baseline_count]
    service = []
    bres = []
    for r in base:
        t1 = time.perf_counter()
        if r["key"] not in meshes_dev:
            m = meshes[r["key"]]
            meshes_dev[r["key"]] = bem.bem_mesh_load(ctx, m.xyz, m.elem)
        kh = _bucket_top(r["k"]) if (kappa > 0.0 and r["green"] == 1) else 0.0
        tk = (r["key"], kh)
        if tk not in trees:
            while trees and ctx.device_bytes()[0] > budget // 2:  # keep the baseline's residency bounded too
                old = next(iter(trees))
                trees.pop(old).close()
            trees[tk] = bem.bem_tree_build(ctx, meshes_dev[r["key"]], B=SERVE_B_HELMHOLTZ if kh > 0 else SERVE_B,
                                           order=8, theta=0.5, kappa=kappa, k_hint=kh)
        else:
            trees[tk] = trees.pop(tk)  # most recently used last
        tree = trees[tk]
        c = _boundary_data(dofs[r["key"]], r)
        cplx = r["green"] == 1
        chid = torch.tensor(c if cplx else c.real, dtype=torch.complex128 if cplx else torch.float64, device="cuda:0")
        phid = torch.empty_like(chid)
        infos = []
        t_b = time.perf_counter()
        for j in range(chid.shape[0]):
            infos += bem.bem_solve(ctx, tree, r["green"], r["k"], chid[j:j + 1], phid[j:j + 1],
                                   precision=bem.BEM_PREC_FP64, max_iters=max_iters,
                                   max_seconds=max(1e-3, max_seconds - (time.perf_counter() - t_b)))
        torch.cuda.synchronize()
        service.append(time.perf_counter() - t1)
        bres.append((0, None, infos, 0.0))
        print(f"{label}: {len(service)} of {len(base)} requests solved one at a time ({service[-1]:.2f} s)",
              file=sys.stderr, flush=True)
    service = np.array(service)
    brhs = sum(r["nrhs"] for r in base)
    out["baseline_requests"] = len(base)
    out["baseline_fp64_solves_per_s"] = brhs / service.sum()
    out["baseline"] = summary(bres)
    out["baseline_service_ms"] = {"p50": float(np.percentile(service, 50) * 1e3),
                                  "p99": float(np.percentile(service, 99) * 1e3)}
    for ol in out["open_loop"]:
        arr = arrivals[:len(base)] / ol["rate_requests_per_s"]
        done, lat = 0.0, []
        for a_, s_ in zip(arr, service):
            done = max(a_, done) + s_
            lat.append(done - a_)
        ol["baseline_latency_ms"] = {"p50": float(np.percentile(lat, 50) * 1e3),
                                     "p99": float(np.percentile(lat, 99) * 1e3),
                                     "note": "FP64 service times, first come first served, same arrivals"}
    # throughput over the same requests on both sides when the baseline covers them all
    out["speedup_solves_per_s"] = out["served_solves_per_s"] / out["baseline_fp64_solves_per_s"]
    for tr in trees.values():
        tr.close()
    for m in meshes_dev.values():
        m.close()
    return out


def cpu_baseline(m, x_np, seconds, fmm=True, B=48, theta=0.5):
    """The oracle (plain FP64 C, OpenMP where it has loops over rows) on the
    headline sphere: a bounded sample of full rows of the direct product of
    the same operator, and (fmm) one whole fast product of the oracle on the
    same tree parameters, timed once."""
    import platform

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
    cpu = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    out = {"value": done / dt, "unit": "unknowns/s", "cores": cores, "kind": "oracle", "cpu": cpu,
           "sample": f"{done} full rows of the direct product A x on the {om.n_dof}-DOF mesh "
                     f"(plain FP64 oracle, {dt:.1f} s)"}
    if fmm:
        print("bench: timing the oracle's fast product (one whole product)", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        T = oracle.OracleTree(om, B=B, theta=theta)
        t1 = time.perf_counter()
        T.fmm_matvec(x_np, oracle.OP_A)
        t2 = time.perf_counter()
        out["fmm"] = {"value": om.n_dof / (t2 - t1), "unit": "unknowns/s", "seconds": t2 - t1,
                      "tree_seconds": t1 - t0,
                      "sample": f"one whole fast product A x of the oracle on the {om.n_dof}-DOF mesh "
                                f"(B = {B}, theta = {theta}, order 8; plain loops, the free term and the "
                                "corrections by direct sums; single-threaded far field, near field and "
                                "corrections over targets on all cores)"}
    return out


if __name__ == "__main__":
    main()
