"""Benchmark of the matrix-free operator action on one MI355X.

Headline workload (the metric's configuration): FP64 Helmholtz and Laplacian
(ncomp 3 -- the paper's vector Laplacian -- and ncomp 1) actions on a 32^3 hex
mesh of the unit cube, vertices perturbed by U(-0.15h, 0.15h), nodes randomly
renumbered, Q_k on GLL nodes for k = 1..6 with (k+1)^3 Gauss points. One step
applies all 18 operators once (y = A x, inputs resident in HBM); `value` is
total DoFs processed per second (GDoF/s).

Also reported (outside the timed steps): per-operator kernel time (mean, min and
median of 5 runs of 20 applies; FP64 also with cold caches), GDoF/s and roofline
fractions in FP64 and FP32, the P1 triangle mass and tet elasticity actions, CG time
to 1e-10 (FP64 Jacobi-CG vs FP32-action iterative refinement, with the error against
a 1e-13 solution), the batched and learned-preconditioner solves, the CPU oracle timed
on a bounded sample of the same workload, and the GPU's difference from the oracle on
that sample.

Output: one compact JSON line on stdout (metric, value, ms_per_step, roofline of the
dominant kernel, cpu_baseline, parity_vs_oracle); the per-operator, simplex, weak-scaled,
CG, batched and learned-preconditioner detail goes to stderr as one line starting with
"detail " (and to --detail-out FILE when given).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--quick]
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12   # 256 CU x 2.4 GHz x 128 FP64 flop/clk (vector FMA)
PEAK_FP32 = 157.3e12  # 256 CU x 2.4 GHz x 256 FP32 flop/clk (packed / MFMA)
PEAK_HBM = 8.0e12     # bytes/s

METRIC = "operator-action GDoF/s + %roofline; CG time-to-1e-10 (FP64 vs FP32-ref/learned)"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_c2_cases(mf, mg, degrees, kinds):
    import torch
    cases = []
    for k in degrees:
        mesh = mg.hex_mesh(32, 0.15, config=1, seed_k=k)
        mfm = mf.Mesh.from_meshgen(mesh)
        for name, kind, ncomp in kinds:
            space = mg.hex_space(mesh, k, ncomp=ncomp, config=1)
            sp = mf.Space(mfm, k, ncomp, space.cell2node, space.nnodes)
            x = mg.uniform(space.ndofs, -1, 1, 1, mg.PURPOSE_X, k)
            ent = {"name": f"{name}-Q{k}", "k": k, "kind": kind, "ncomp": ncomp, "ndofs": space.ndofs,
                   "space": space, "ops": {}}
            for prec in (mf.F64, mf.F32):
                op = mf.Operator(sp, kind, prec)
                xt = torch.tensor(x, device="cuda", dtype=op.torch_dtype)
                yt = torch.empty_like(xt)
                ent["ops"][prec] = (op, xt, yt)
            cases.append(ent)
            log(f"  built {ent['name']} ({space.ndofs} dofs)")
    return cases


def time_kernel(op, x, y, reps):
    """Average duration of the action's cell-kernel launches alone, internal numbering:
    an overwrite apply where it runs no clearing pass (as in the headline step), else an
    accumulating apply (the same launches without the clearing pass)."""
    import torch
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    nc = op.info["ncells"]
    if op.info["clears_output"]:
        run = lambda: op.apply_range_internal(0, nc, x, y, accumulate=True)
    else:
        run = lambda: op.apply_internal(x, y)
    y.zero_()
    run()
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        run()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def time_kernel_cold(op, x, y, flush, reps=5):
    """The launches of time_kernel with cold caches: each apply follows a write of
    `flush` (512 MiB, more than the 4 MiB L2 of every XCD and the 256 MiB Infinity
    Cache), timed on its own with HIP events; the mean over reps."""
    import torch
    s = torch.cuda.current_stream()
    nc = op.info["ncells"]
    if op.info["clears_output"]:
        run = lambda: op.apply_range_internal(0, nc, x, y, accumulate=True)
    else:
        run = lambda: op.apply_internal(x, y)
    run()
    tot = 0.0
    for _ in range(reps):
        flush.fill_(1.0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        run()
        e1.record(s)
        e1.synchronize()
        tot += e0.elapsed_time(e1) * 1e-3
    return tot / reps


def roof(op, t, prec):
    F, B = op.info["flops_per_apply"], op.info["bytes_per_apply"]
    P = PEAK_FP64 if prec == 0 else PEAK_FP32
    t_f, t_b = F / P, B / PEAK_HBM
    bound = "alu" if t_f >= t_b else "hbm"
    return {"bound": bound, "flops": F, "bytes": B, "t_roof_s": max(t_f, t_b), "frac": max(t_f, t_b) / t,
            "tflops": F / t / 1e12, "gbs": B / t / 1e9}


PROFILE = os.path.join(ROOT, "profiles", "hex_apply_laplacian3_q6_fp64_32cube.md")


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter summary,
    or None when the kernel source has changed since the counters were taken."""
    import hashlib
    try:
        kv = {}
        for line in open(PROFILE):
            parts = line.strip().split(": ", 1)
            if len(parts) == 2:
                kv[parts[0]] = parts[1]
        # the sources the kernel is built from, hashed as one concatenation in order
        h = hashlib.sha256()
        for src in kv["kernel_source"].split(","):
            h.update(open(os.path.join(ROOT, src.strip()), "rb").read())
        if h.hexdigest() != kv["kernel_source_sha256"]:
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(mg, cases, budget_s=30.0):
    """The oracle (dense, FP64, all host cores) on a bounded sample: a contiguous
    slice of cells of every headline operator, scaled to GDoF/s by the slice fraction.
    Outside the timed oracle calls, the GPU applies the same cell range to the same x
    (both precisions); the largest relative max-norm difference is returned as well."""
    import oracle
    import torch
    nthreads = oracle.default_threads()
    tot_dofs, tot_t = 0.0, 0.0
    frac = 0.75  # about 11 s of oracle work on 16 host threads
    samples = []
    err = {0: 0.0, 1: 0.0}
    for ent in cases:
        sp = ent["space"]
        orc = oracle.OracleOp(sp, ent["kind"])
        x = mg.uniform(sp.ndofs, -1, 1, 1, mg.PURPOSE_X, ent["k"])
        nc = orc.ncells
        c1 = max(1, int(nc * frac))
        t0 = time.perf_counter()
        ref = orc.apply(x, cells=(0, c1), nthreads=nthreads)
        dt = time.perf_counter() - t0
        for prec, (op, xt, yt) in ent["ops"].items():
            y = op.apply_range(0, c1, xt, yt).double().cpu().numpy()
            err[prec] = max(err[prec], float(np.abs(y - ref).max() / np.abs(ref).max()))
        tot_dofs += ent["ndofs"] * (c1 / nc)
        tot_t += dt
        samples.append(ent["name"])
        if tot_t > budget_s:
            break
    cpu = {"value": tot_dofs / tot_t / 1e9, "unit": "GDoF/s", "cores": nthreads, "kind": "oracle",
           "sample": f"cells [0, {frac:g} ncells) of each of {len(samples)} headline operators "
                     f"({samples[0]}..{samples[-1]}), dofs scaled by the cell fraction; "
                     f"{tot_t:.1f} s of CPU work"}
    parity = {"operators": len(samples), "cells": f"[0, {frac:g} ncells)",
              "max_rel_error_fp64": err[0], "max_rel_error_fp32": err[1],
              "tolerance_fp64": 1e-12, "tolerance_fp32": 1e-5}
    return cpu, parity


def bench_simplex(mf, mg, reps=20):
    """P1 triangle mass with a nodal coefficient (64x64x2 triangles, and a weak-scaled
    2048x2048x2 mesh for the bandwidth figure; patch scatter by default there, atomic
    for comparison) and vector P2/P3 tet elasticity (48^3 x 6 Kuhn tets perturbed
    +-0.2h, renumbered, lambda 1, mu 0.5) in FP64 and FP32 (MFMA contractions; patch
    scatter by default, coloured launches for comparison); the one-component tet
    operators and the hyperelastic tangent on the same mesh; degrees 4-6 on smaller
    meshes. Per operator: kernel time (every launch of one apply), GDoF/s, roofline
    fraction."""
    import torch
    out = {}
    for m, tag, sc in ((64, "tri_p1_mass_64", mf.SCATTER_AUTO),
                       (2048, "tri_p1_mass_2048_weak_scaled", mf.SCATTER_AUTO),
                       (2048, "tri_p1_mass_2048_weak_scaled_atomic_scatter", mf.SCATTER_ATOMIC)):
        mesh = mg.tri_mesh(m)
        space = mg.tri_p1_space(mesh)
        c = mg.uniform(mesh.nverts, 0.5, 1.5, 0, mg.PURPOSE_COEF)
        sp = mf.Space.from_meshgen(space)
        op = mf.Operator(sp, mf.MASS, mf.F64, vertex_coef=c, scatter=sc)
        x = torch.tensor(mg.uniform(space.ndofs, -1, 1, 0, mg.PURPOSE_X), device="cuda")
        y = torch.empty_like(x)
        t = time_kernel(op, x, y, reps)
        r = roof(op, t, 0)
        out[tag] = {"cells": mesh.ncells, "ndofs": space.ndofs, "us": t * 1e6, "gdofs": space.ndofs / t / 1e9,
                    "bound": r["bound"], "frac": r["frac"], "gbs": r["gbs"]}
        log(f"  {tag}: {json.dumps(out[tag])}")
    mesh = mg.tet_mesh(48, 0.2, config=2)
    for k in (2, 3):
        space = mg.tet_space(mesh, k, config=2)
        sp = mf.Space.from_meshgen(space)
        x = mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_X, k)
        for prec, ptag, sc in ((mf.F64, "fp64", mf.SCATTER_AUTO), (mf.F32, "fp32", mf.SCATTER_AUTO),
                               (mf.F64, "fp64_coloured_scatter", mf.SCATTER_COLOURED),
                               (mf.F32, "fp32_coloured_scatter", mf.SCATTER_COLOURED)):
            op = mf.Operator(sp, mf.ELASTICITY, prec, lam=1.0, mu=0.5, scatter=sc)
            xt = torch.tensor(x, device="cuda", dtype=op.torch_dtype)
            yt = torch.empty_like(xt)
            t = time_kernel(op, xt, yt, reps)
            F, B = op.info["flops_per_apply"], op.info["bytes_per_apply"]
            P = PEAK_FP64 if prec == mf.F64 else PEAK_FP32
            tag = f"tet_elasticity_p{k}_{ptag}"
            out[tag] = {"cells": mesh.ncells, "ndofs": space.ndofs, "us": t * 1e6, "gdofs": space.ndofs / t / 1e9,
                        "launches": op.info["cell_launches"],
                        "bound": "mfma", "tflops": F / t / 1e12,
                        "frac": max(F / P, B / PEAK_HBM) / t, "gbs": B / t / 1e9}
            log(f"  {tag}: {json.dumps(out[tag])}")
            del op, xt, yt
        del sp, space
    # P2 / P3 triangles (lane per cell), 1024 x 1024 x 2 cells
    tmesh = mg.tri_mesh(1024, 0.2, config=0)
    for k, kind, name, nc in ((2, mf.HELMHOLTZ, "helmholtz", 1), (3, mf.LAPLACIAN, "laplacian", 1),
                              (2, mf.ELASTICITY, "elasticity", 2)):
        space = mg.tri_space(tmesh, k, ncomp=nc)
        sp = mf.Space.from_meshgen(space)
        x = mg.uniform(space.ndofs, -1, 1, 0, mg.PURPOSE_X, k)
        for prec, ptag in ((mf.F64, "fp64"), (mf.F32, "fp32")):
            op = mf.Operator(sp, kind, prec)
            xt = torch.tensor(x, device="cuda", dtype=op.torch_dtype)
            yt = torch.empty_like(xt)
            t = time_kernel(op, xt, yt, reps)
            r = roof(op, t, prec)
            tag = f"tri_{name}_p{k}_{ptag}"
            out[tag] = {"cells": tmesh.ncells, "ndofs": space.ndofs, "us": t * 1e6, "gdofs": space.ndofs / t / 1e9,
                        "launches": op.info["cell_launches"], "qp": op.info["nqp"], "bound": r["bound"],
                        "frac": r["frac"], "gbs": r["gbs"], "tflops": r["tflops"]}
            log(f"  {tag}: {json.dumps(out[tag])}")
            del op, xt, yt
        del sp, space
    del tmesh
    # elasticity and the hyperelastic tangent (u0 = 0.3 U[-1, 1]) on Q2 / Q4 hexahedra
    # (32^3 cells, one workgroup per cell)
    hmesh = mg.hex_mesh(32, 0.15, config=1)
    for k in (2, 4):
        space = mg.hex_space(hmesh, k, ncomp=3)
        sp = mf.Space.from_meshgen(space)
        x = mg.uniform(space.ndofs, -1, 1, 1, mg.PURPOSE_X, k)
        u0 = 0.3 * mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_COEF, k)
        for (prec, ptag), (kind, kname) in itertools.product(((mf.F64, "fp64"), (mf.F32, "fp32")),
                                                              ((mf.ELASTICITY, "elasticity"),
                                                               (mf.HYPERELASTIC, "hyperelastic"))):
            op = mf.Operator(sp, kind, prec, u0=u0 if kind == mf.HYPERELASTIC else None)
            xt = torch.tensor(x, device="cuda", dtype=op.torch_dtype)
            yt = torch.empty_like(xt)
            t = time_kernel(op, xt, yt, reps)
            r = roof(op, t, prec)
            tag = f"hex_{kname}_q{k}_{ptag}"
            out[tag] = {"cells": hmesh.ncells, "ndofs": space.ndofs, "us": t * 1e6, "gdofs": space.ndofs / t / 1e9,
                        "launches": op.info["cell_launches"], "qp": op.info["nqp"], "bound": r["bound"],
                        "frac": r["frac"], "gbs": r["gbs"], "tflops": r["tflops"]}
            log(f"  {tag}: {json.dumps(out[tag])}")
            del op, xt, yt
        del sp, space
    del hmesh
    # Q_k quadrilaterals (2D sum factorisation, lane per point), 1024 x 1024 cells
    qmesh = mg.quad_mesh(1024, 0.25, config=0)
    for k, kind, name, nc in ((2, mf.HELMHOLTZ, "helmholtz", 1), (6, mf.LAPLACIAN, "laplacian", 1),
                              (2, mf.ELASTICITY, "elasticity", 2)):
        space = mg.quad_space(qmesh, k, ncomp=nc)
        sp = mf.Space.from_meshgen(space)
        x = mg.uniform(space.ndofs, -1, 1, 0, mg.PURPOSE_X, k)
        for prec, ptag in ((mf.F64, "fp64"), (mf.F32, "fp32")):
            op = mf.Operator(sp, kind, prec)
            xt = torch.tensor(x, device="cuda", dtype=op.torch_dtype)
            yt = torch.empty_like(xt)
            t = time_kernel(op, xt, yt, reps)
            r = roof(op, t, prec)
            tag = f"quad_{name}_q{k}_{ptag}"
            out[tag] = {"cells": qmesh.ncells, "ndofs": space.ndofs, "us": t * 1e6, "gdofs": space.ndofs / t / 1e9,
                        "launches": op.info["cell_launches"], "qp": op.info["nqp"], "bound": r["bound"],
                        "frac": r["frac"], "gbs": r["gbs"], "tflops": r["tflops"]}
            log(f"  {tag}: {json.dumps(out[tag])}")
            del op, xt, yt
        del sp, space
    del qmesh
    # one-component operators on the same tets (dense tabulation, lane per cell)
    for k, kind, name in ((1, mf.LAPLACIAN, "laplacian"), (2, mf.HELMHOLTZ, "helmholtz"),
                          (2, mf.LAPLACIAN, "laplacian"), (3, mf.LAPLACIAN, "laplacian"),
                          (3, mf.HELMHOLTZ, "helmholtz")):
        space = mg.tet_space(mesh, k, ncomp=1, config=2)
        sp = mf.Space.from_meshgen(space)
        x = mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_X, k)
        for prec, ptag in ((mf.F64, "fp64"), (mf.F32, "fp32")):
            op = mf.Operator(sp, kind, prec)
            xt = torch.tensor(x, device="cuda", dtype=op.torch_dtype)
            yt = torch.empty_like(xt)
            t = time_kernel(op, xt, yt, reps)
            r = roof(op, t, prec)
            tag = f"tet_{name}_p{k}_{ptag}"
            out[tag] = {"cells": mesh.ncells, "ndofs": space.ndofs, "us": t * 1e6, "gdofs": space.ndofs / t / 1e9,
                        "launches": op.info["cell_launches"], "qp": op.info["nqp"], "bound": r["bound"],
                        "frac": r["frac"], "gbs": r["gbs"], "tflops": r["tflops"]}
            log(f"  {tag}: {json.dumps(out[tag])}")
            del op, xt, yt
        del sp, space
    # the paper's hyperelasticity operator: the St-Venant-Kirchhoff tangent at a
    # displacement u0 = 0.3 U[-1,1], P1-P3 on the same mesh (P3: 125 points per cell)
    for k in (1, 2, 3):
        space = mg.tet_space(mesh, k, config=2)
        sp = mf.Space.from_meshgen(space)
        x = mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_X, k)
        u0 = 0.3 * mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_COEF, k)
        for prec, ptag in ((mf.F64, "fp64"), (mf.F32, "fp32")):
            op = mf.Operator(sp, mf.HYPERELASTIC, prec, lam=1.0, mu=0.5, u0=u0)
            xt = torch.tensor(x, device="cuda", dtype=op.torch_dtype)
            yt = torch.empty_like(xt)
            t = time_kernel(op, xt, yt, reps)
            F, B = op.info["flops_per_apply"], op.info["bytes_per_apply"]
            P = PEAK_FP64 if prec == mf.F64 else PEAK_FP32
            tag = f"tet_hyperelastic_p{k}_{ptag}"
            out[tag] = {"cells": mesh.ncells, "ndofs": space.ndofs, "us": t * 1e6, "gdofs": space.ndofs / t / 1e9,
                        "launches": op.info["cell_launches"], "qp": op.info["nqp"],
                        "bound": "mfma", "tflops": F / t / 1e12,
                        "frac": max(F / P, B / PEAK_HBM) / t, "gbs": B / t / 1e9}
            log(f"  {tag}: {json.dumps(out[tag])}")
            del op, xt, yt
        del sp, space
    del mesh
    # degrees 4-6 (the dense kernel: a workgroup per block of cells, the points in
    # chunks), 24^3 x 6 tets and 512^2 x 2 triangles, coloured scatter
    for cell, k, kind, name, nc in (("tet", 4, mf.LAPLACIAN, "laplacian", 1), ("tet", 4, mf.ELASTICITY, "elasticity", 3),
                                    ("tet", 6, mf.LAPLACIAN, "laplacian", 1), ("tri", 6, mf.HELMHOLTZ, "helmholtz", 1)):
        if cell == "tet":
            smesh = mg.tet_mesh(24, 0.2, config=2)
            space = mg.tet_space(smesh, k, ncomp=nc, config=2)
        else:
            smesh = mg.tri_mesh(512, 0.2, config=0)
            space = mg.tri_space(smesh, k, ncomp=nc)
        sp = mf.Space.from_meshgen(space)
        x = mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_X, k)
        for prec, ptag in ((mf.F64, "fp64"), (mf.F32, "fp32")):
            op = mf.Operator(sp, kind, prec, lam=1.0, mu=0.5)
            xt = torch.tensor(x, device="cuda", dtype=op.torch_dtype)
            yt = torch.empty_like(xt)
            t = time_kernel(op, xt, yt, 5)
            r = roof(op, t, prec)
            tag = f"{cell}_{name}_p{k}_{ptag}"
            out[tag] = {"cells": smesh.ncells, "ndofs": space.ndofs, "us": t * 1e6, "gdofs": space.ndofs / t / 1e9,
                        "launches": op.info["cell_launches"], "qp": op.info["nqp"], "bound": r["bound"],
                        "frac": r["frac"], "gbs": r["gbs"], "tflops": r["tflops"]}
            log(f"  {tag}: {json.dumps(out[tag])}")
            del op, xt, yt
        del sp, space, smesh
    return out


# The paper's Table 2 (operator characteristics on its CPUs): arithmetic intensity
# (FLOP/byte under perfect caching), D (loop trip count over degrees of freedom; per
# direction on quad/hex) and Q (over quadrature points; per direction on quad/hex) for
# P1..P6, per operator and cell. Quoted for comparison with the same quantities of the
# operators built here.
TABLE2 = {
    ("mass", "tri"): [(1.2, 3, 3), (1.7, 6, 6), (3.0, 10, 12), (5.6, 15, 25), (7.5, 21, 36), (9.7, 28, 49)],
    ("mass", "quad"): [(4.7, 2, 3), (3.9, 3, 4), (3.9, 4, 5), (3.9, 5, 6), (3.9, 6, 7), (4.1, 7, 8)],
    ("mass", "tet"): [(2.7, 4, 4), (5.9, 10, 14), (8.7, 20, 24), (39.2, 35, 125), (55.9, 56, 216), (81.2, 84, 343)],
    ("mass", "hex"): [(16.9, 2, 3), (10.8, 3, 4), (8.5, 4, 5), (7.4, 5, 6), (7.0, 6, 7), (6.9, 7, 8)],
    ("helmholtz", "tri"): [(1.8, 3, 3), (5.7, 6, 6), (9.6, 10, 12), (17.8, 15, 25), (23.3, 21, 36), (29.9, 28, 49)],
    ("helmholtz", "quad"): [(10.7, 2, 3), (10.6, 3, 4), (10.5, 4, 5), (10.5, 5, 6), (10.4, 6, 7), (10.9, 7, 8)],
    ("helmholtz", "tet"): [(3.9, 4, 4), (27.3, 10, 14), (37.5, 20, 24), (164.1, 35, 125), (230.1, 56, 216),
                           (331.4, 84, 343)],
    ("helmholtz", "hex"): [(45.5, 2, 3), (34.9, 3, 4), (27.9, 4, 5), (24.5, 5, 6), (23.1, 6, 7), (22.7, 7, 8)],
    ("laplacian", "tri"): [(0.5, 3, 1), (2.7, 6, 3), (4.0, 10, 6), (6.9, 15, 12), (12.6, 21, 25), (16.8, 28, 36)],
    ("laplacian", "quad"): [(7.9, 2, 3), (8.7, 3, 4), (8.4, 4, 5), (8.3, 5, 6), (8.2, 6, 7), (8.6, 7, 8)],
    ("laplacian", "tet"): [(1.9, 4, 1), (10.4, 10, 4), (24.0, 20, 14), (31.5, 35, 24), (124.3, 56, 125),
                           (189.3, 84, 216)],
    ("laplacian", "hex"): [(37.8, 2, 3), (27.1, 3, 4), (21.6, 4, 5), (19.2, 5, 6), (18.4, 6, 7), (18.3, 7, 8)],
    ("elasticity", "tri"): [(0.5, 3, 1), (3.0, 6, 3), (4.4, 10, 6), (7.3, 15, 12), (13.2, 21, 25), (17.4, 28, 36)],
    ("elasticity", "quad"): [(10.2, 2, 3), (10.2, 3, 4), (9.5, 4, 5), (9.2, 5, 6), (9.0, 6, 7), (9.3, 7, 8)],
    ("elasticity", "tet"): [(1.9, 4, 1), (11.6, 10, 4), (25.6, 20, 14), (32.7, 35, 24), (127.5, 56, 125),
                            (192.6, 84, 216)],
    ("elasticity", "hex"): [(48.0, 2, 3), (31.8, 3, 4), (24.4, 4, 5), (21.3, 5, 6), (20.1, 6, 7), (19.8, 7, 8)],
    ("hyperelasticity", "tet"): [(1.7, 4, 1), (63.2, 10, 14), (313.8, 20, 125), (600.0, 35, 343),
                                 (915.2, 56, 729), (1428.3, 84, 1331)],
}


def table2(mf, mg):
    """D, Q and arithmetic intensity of every operator built here, beside the paper's
    Table 2 row for the same operator, cell and degree. Ours: D = nodes per cell (per
    direction on quad/hex), Q = quadrature points (per direction on quad/hex), AI =
    the algorithmic flops / algorithmic HBM bytes of one FP64 action on a small mesh
    (counted as in the roofline: x read and y written once, map, geometry); the paper
    counts per element with its own caching model, so the AIs are not the same measure.
    Hex and quad are built with k+1 and, where the kernels allow it, the paper's k+2
    points per direction. Nothing is timed."""
    meshes = {"tri": mg.tri_mesh(16, 0.2, config=0), "quad": mg.quad_mesh(16, 0.25, config=0),
              "tet": mg.tet_mesh(6, 0.2, config=2), "hex": mg.hex_mesh(8, 0.15, config=1)}
    kinds = {"mass": mf.MASS, "helmholtz": mf.HELMHOLTZ, "laplacian": mf.LAPLACIAN, "elasticity": mf.ELASTICITY,
             "hyperelasticity": mf.HYPERELASTIC}
    dim = {"tri": 2, "quad": 2, "tet": 3, "hex": 3}
    rows = []
    for (opname, cell), ref in TABLE2.items():
        for k in range(1, 7):
            ncomp = dim[cell] if opname in ("laplacian", "elasticity", "hyperelasticity") else 1
            mesh = meshes[cell]
            row = {"op": opname, "cell": cell, "k": k, "paper": {"AI": ref[k - 1][0], "D": ref[k - 1][1],
                                                              "Q": ref[k - 1][2]}}
            for q_extra in ((0, 1) if cell in ("quad", "hex") else (0,)):
                tag = "ours" if q_extra == 0 else "ours_q_k+2"
                try:
                    if cell == "tri":
                        space = mg.tri_space(mesh, k, ncomp=ncomp) if k > 1 or ncomp > 1 else mg.tri_p1_space(mesh)
                    elif cell == "quad":
                        space = mg.quad_space(mesh, k, ncomp=ncomp)
                    elif cell == "tet":
                        space = mg.tet_space(mesh, k, ncomp=ncomp, config=2)
                    else:
                        space = mg.hex_space(mesh, k, ncomp=ncomp, config=1)
                    kw = {}
                    if opname == "hyperelasticity":
                        kw["u0"] = 0.3 * mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_COEF, k)
                    op = mf.Operator(mf.Space.from_meshgen(space), kinds[opname], mf.F64,
                                     nq1d=(k + 2 if q_extra else 0), **kw)
                    inf = op.info
                    tensor = cell in ("quad", "hex")
                    row[tag] = {"AI": inf["flops_per_apply"] / inf["bytes_per_apply"],
                                "D": k + 1 if tensor else inf["dofs_per_cell"],
                                "Q": inf["nq1d"] if tensor else inf["nqp"]}
                    del op
                except Exception as ex:  # not built for this combination
                    row[tag] = {"not_built": str(ex)[:80]}
            rows.append(row)
    return rows


def bench_hex_q(mf, cases, reps=20):
    """The paper's hex rule, k+2 Gauss points per direction (Table 2's Q), on the
    headline meshes: FP64 and FP32, every operator of the headline sweep, Q1..Q6,
    beside the same operators with k+1 points (the headline rule)."""
    out = {}
    for ent in cases:
        sp = ent["ops"][mf.F64][0].space
        row = {"ndofs": ent["ndofs"]}
        for prec, tag in ((mf.F64, "fp64"), (mf.F32, "fp32")):
            _, x, y = ent["ops"][prec]
            op = mf.Operator(sp, ent["kind"], prec, nq1d=ent["k"] + 2)
            t = float(np.mean([time_kernel(op, x, y, reps) for _ in range(3)]))
            r = roof(op, t, prec)
            row[tag] = {"us": t * 1e6, "gdofs": ent["ndofs"] / t / 1e9, "frac": r["frac"], "bound": r["bound"],
                        "tflops": r["tflops"]}
            del op
        out[ent["name"] + "_q_k+2"] = row
        log(f"  {ent['name']} k+2 points: fp64 {row['fp64']['us']:.1f} us {row['fp64']['gdofs']:.1f} GDoF/s | "
            f"fp32 {row['fp32']['us']:.1f} us {row['fp32']['gdofs']:.1f} GDoF/s")
    return out


def bench_weak(mf, mg, reps=20):
    """The bandwidth-bound low-degree hex actions at a weak-scaled size (128^3 cells
    instead of 32^3, same perturbation and random renumbering): FP64 Helmholtz and
    scalar Laplacian, Q1 and Q2."""
    import torch
    out = {}
    mesh = mg.hex_mesh(128, 0.15, config=1, seed_k=1)
    for k in (1, 2):
        space = mg.hex_space(mesh, k, config=1)
        sp = mf.Space.from_meshgen(space)
        x = torch.tensor(mg.uniform(space.ndofs, -1, 1, 1, mg.PURPOSE_X, k), device="cuda")
        y = torch.empty_like(x)
        for name, kind in (("helmholtz", mf.HELMHOLTZ), ("laplacian1", mf.LAPLACIAN)):
            op = mf.Operator(sp, kind, mf.F64)
            t = time_kernel(op, x, y, reps)
            r = roof(op, t, 0)
            tag = f"{name}-Q{k}_128cube"
            # design-independent minimum: x and y once, the int32 cell map, FP64 vertex
            # coordinates once (the kernels read 24 stored geometry values per cell instead)
            bmin = 2.0 * space.ndofs * 8 + 4.0 * space.cell2node.shape[1] * mesh.ncells + 24.0 * mesh.nverts
            out[tag] = {"cells": mesh.ncells, "ndofs": space.ndofs, "us": t * 1e6, "gdofs": space.ndofs / t / 1e9,
                        "bound": r["bound"], "frac": r["frac"], "gbs": r["gbs"], "tflops": r["tflops"],
                        "bmin_bytes": bmin, "frac_bmin": bmin / t / PEAK_HBM}
            log(f"  {tag}: {json.dumps(out[tag])}")
            del op
        del sp, space
    return out


def bench_cg(mf, mg, k=3, m=32):
    """Time to 1e-10 relative residual: FP64 Jacobi-CG vs FP32-action refinement (Helmholtz)."""
    import torch
    mesh = mg.hex_mesh(m, 0.15, config=3, seed_k=k)
    space = mg.hex_space(mesh, k, config=3)
    sp = mf.Space.from_meshgen(space)
    A64 = mf.Operator(sp, mf.HELMHOLTZ, mf.F64)
    A32 = mf.Operator(sp, mf.HELMHOLTZ, mf.F32)
    M = mf.JacobiPrecond(A64)
    b = torch.tensor(mg.uniform(space.ndofs, -1, 1, 3, mg.PURPOSE_RHS, k), device="cuda")
    out = {"problem": f"Helmholtz Q{k}, {m}^3 perturbed renumbered hex, {space.ndofs} dofs, Jacobi"}
    xref = torch.zeros_like(b)  # reference: FP64 Jacobi-CG to 1e-13 (untimed)
    mf.cg_solve(A64, b, xref, precond=M, rtol=1e-13, maxit=20000, raise_on_error=False)
    for name, a32 in (("fp64", None), ("fp32_refined", A32)):
        x = torch.zeros_like(b)
        mf.cg_solve(A64, b, x, A32=a32, precond=M, rtol=1e-10)  # warm (graph capture, caches)
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = mf.cg_solve(A64, b, x, A32=a32, precond=M, rtol=1e-10)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = {"seconds": dt, "iterations": info["inner_iterations"], "outer": info["outer_iterations"],
                     "rel_residual": info["rel_residual"],
                     "rel_error_vs_1e-13_solution": float((x - xref).norm() / xref.norm())}
    return out


def bench_c4(mf, mg, nsys=64, seed=0, m_lo=8, m_hi=40):
    """64 Helmholtz systems on hex meshes m ~ U{m_lo..m_hi}^3, Q_k with k ~ U{2..5},
    b ~ U[-1,1]: FP32-action batched CG with FP64 refinement to 1e-10 (autotuned launch)
    vs the same batch in FP64 vs one FP64 Jacobi-CG solve after another."""
    import tempfile

    import torch
    r = np.random.default_rng([4, 9, seed])
    ms, ks = r.integers(m_lo, m_hi + 1, size=nsys), r.integers(2, 6, size=nsys)
    sy = []
    for i in range(nsys):
        mesh = mg.hex_mesh(int(ms[i]), 0.15, config=3, seed_k=100 + i)
        space = mg.hex_space(mesh, int(ks[i]), config=3, seed_k=100 + i)
        sp = mf.Space.from_meshgen(space)
        A64 = mf.Operator(sp, mf.HELMHOLTZ, mf.F64)
        A32 = mf.Operator(sp, mf.HELMHOLTZ, mf.F32)
        M = mf.JacobiPrecond(A64)
        b = torch.tensor(mg.uniform(space.ndofs, -1, 1, 3, mg.PURPOSE_RHS, 100 + i), device="cuda")
        sy.append((A64, A32, M, b))
    ndofs = sum(int(s[3].numel()) for s in sy)
    out = {"systems": nsys, "total_dofs": ndofs, "mesh_m": [int(v) for v in ms], "degree": [int(v) for v in ks]}
    # reference solutions: FP64 Jacobi-CG to 1e-13 (untimed)
    xref = [torch.zeros_like(s[3]) for s in sy]
    for (A64, A32, M, b), x in zip(sy, xref):
        mf.cg_solve(A64, b, x, precond=M, rtol=1e-13, maxit=20000, raise_on_error=False)

    def max_err(xs):
        return max(float((x - xr).norm() / xr.norm()) for x, xr in zip(xs, xref))

    cache = os.path.join(tempfile.gettempdir(), "mf_batch_tuning.txt")
    for name, refined in (("batched_fp32_refined", True), ("batched_fp64", False)):
        xs = [torch.zeros_like(s[3]) for s in sy]
        B = mf.Batch([s[0] for s in sy], [s[3] for s in sy], xs, A32=[s[1] for s in sy] if refined else None,
                     M=[s[2] for s in sy])
        t0 = time.perf_counter()
        tune = B.autotune(cache)
        t_tune = time.perf_counter() - t0
        B.solve(rtol=1e-10)  # warm-up (graph capture)
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos, rc = B.solve(rtol=1e-10)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = {"seconds": dt, "rc": rc, "max_rel_residual": max(i["rel_residual"] for i in infos),
                     "max_inner_iterations": max(i["inner_iterations"] for i in infos),
                     "max_outer": max(i["outer_iterations"] for i in infos),
                     "max_rel_error_vs_1e-13_solution": max_err(xs),
                     "tuning_items_per_grid": list(tune), "autotune_seconds": t_tune}
        del B
    xs = [torch.zeros_like(s[3]) for s in sy]
    for (A64, A32, M, b), x in zip(sy, xs):  # warm
        mf.cg_solve(A64, b, x, precond=M, rtol=1e-10)
    for x in xs:
        x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [mf.cg_solve(A64, b, x, precond=M, rtol=1e-10) for (A64, A32, M, b), x in zip(sy, xs)]
    torch.cuda.synchronize()
    out["sequential_fp64"] = {"seconds": time.perf_counter() - t0,
                              "max_rel_residual": max(i["rel_residual"] for i in res),
                              "max_iterations": max(i["inner_iterations"] for i in res),
                              "max_rel_error_vs_1e-13_solution": max_err(xs)}
    return out


def bench_c5(mf, mg, m=64, k=3, channels=8, levels=7, steps=800, lr=1e-3, train_rhs=2, seed=0):
    """Variable-coefficient Poisson, Q3 on 64^3 hex (193^3 = 7,189,057 dofs), kappa =
    exp(GRF), homogeneous Dirichlet, b = M f: time to 1e-10 with Jacobi-CG (FP64, and
    FP32-action refinement) against flexible CG with the learned preconditioner
    (FP32-action refinement, and FP64). The network is trained on the energy loss
    over residuals of Jacobi-CG iterates of other right-hand sides (full lattice,
    one residual per Adam step); harvest and training are timed separately."""
    import torch
    t_setup = time.perf_counter()
    mesh = mg.hex_mesh(m, 0.15, config=5, seed_k=seed)
    space = mg.hex_space(mesh, k, config=5, seed_k=seed)
    kappa = np.exp(mg.gaussian_random_field(mesh.vert_ijk, m, config=5))
    bnd = space.boundary_nodes()
    mask = np.zeros(space.nnodes, np.uint8)
    mask[bnd] = 1
    G = m * k + 1
    ijk = space.node_ijk
    node_grid = (ijk[:, 0] + G * (ijk[:, 1] + G * ijk[:, 2])).astype(np.int32)
    sp = mf.Space.from_meshgen(space)
    A64 = mf.Operator(sp, mf.POISSON, mf.F64, vertex_coef=kappa, dirichlet=mask)
    A32 = mf.Operator(sp, mf.POISSON, mf.F32, vertex_coef=kappa, dirichlet=mask)
    Mass = mf.Operator(sp, mf.MASS, mf.F64, dirichlet=mask)
    J = mf.JacobiPrecond(A64)

    def rhs(i):
        f = mg.uniform(space.ndofs, -1, 1, 5, mg.PURPOSE_RHS, i)
        f[bnd] = 0.0
        return Mass.apply(torch.tensor(f, device="cuda"))

    out = {"problem": f"variable-kappa Poisson Q{k}, {m}^3 perturbed renumbered hex, {space.ndofs} dofs, "
                      "Dirichlet, kappa = exp(GRF, l=0.1)", "setup_seconds": time.perf_counter() - t_setup}
    net = mf.CNN(channels, levels, mf.cnn_initial_weights(channels, levels, seed=seed))
    M = mf.LearnedPrecond(A64, net, (G, G, G), node_grid)
    # training residuals: r_j = b - A x_j of Jacobi-CG iterates x_j for right-hand sides
    # b = A e with e uniform noise on the free DoFs: the first residual (x_0 = 0) is the
    # image of an error with every frequency, the later ones of smoother errors, so the
    # residuals span the whole spectrum the preconditioner must handle
    g = np.random.default_rng([5, 7, seed])
    snaps = sorted(set(int(round(1.3 ** i)) for i in range(0, 30) if round(1.3 ** i) <= 1500))
    free = torch.ones(space.ndofs, dtype=torch.float64, device="cuda")
    free[torch.tensor(bnd, device="cuda").long()] = 0.0

    def rhs_noise(i):
        e = torch.tensor(np.random.default_rng([5, 8, seed, i]).uniform(-1, 1, space.ndofs), device="cuda")
        return A64.apply(e * free)

    t0 = time.perf_counter()
    R = []
    for i in range(train_rhs):
        b = rhs_noise(i)
        R.append(b.clone())
        for j in snaps:
            xj = torch.zeros_like(b)
            mf.cg_solve(A64, b, xj, precond=J, rtol=1e-14, maxit=j, raise_on_error=False)
            R.append(b - A64.apply(xj))
        log(f"  c5 training rhs {i}: {len(snaps) + 1} residuals")
    R = torch.stack(R)
    torch.cuda.synchronize()
    out["harvest_seconds"] = time.perf_counter() - t0
    out["samples"] = int(R.shape[0])
    t0 = time.perf_counter()
    losses = net.train_energy(M, A64, R, g.integers(0, R.shape[0], size=steps), lr=lr)
    out["train_seconds"] = time.perf_counter() - t0
    out["train"] = {"loss": "energy", "rhs": "A e, e ~ U[-1,1] on free dofs", "steps": steps, "lr": lr,
                    "channels": channels, "levels": levels,
                    "loss_first": float(np.mean(losses[:10])), "loss_last": float(np.mean(losses[-50:]))}
    log(f"  c5 trained {steps} steps: energy loss {out['train']['loss_first']:.4f} -> {out['train']['loss_last']:.4f}")
    del R
    torch.cuda.empty_cache()
    b = rhs(0)
    # reference solution: FP64 Jacobi-CG to 1e-13 (untimed)
    xref = torch.zeros_like(b)
    mf.cg_solve(A64, b, xref, precond=J, rtol=1e-13, maxit=200000, raise_on_error=False)
    for name, a32, prec in (("jacobi_fp64", None, J), ("jacobi_fp32_refined", A32, J),
                            ("learned_fp32_refined", A32, M), ("learned_fp64", None, M)):
        x = torch.zeros_like(b)
        mf.cg_solve(A64, b, x, A32=a32, precond=prec, rtol=1e-10, maxit=200000)  # warm (graph capture)
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = mf.cg_solve(A64, b, x, A32=a32, precond=prec, rtol=1e-10, maxit=200000)
        torch.cuda.synchronize()
        out[name] = {"seconds": time.perf_counter() - t0, "iterations": info["inner_iterations"],
                     "outer": info["outer_iterations"], "fallbacks": info["fallbacks"],
                     "rel_residual": info["rel_residual"],
                     "rel_error_vs_1e-13_solution": float((x - xref).norm() / xref.norm())}
        log(f"  c5 {name}: {json.dumps(out[name])}")
    return out


def profile_kernel(mf, mg):
    """The dominant kernel of the headline step (FP64 3-component Laplacian, Q6, 32^3)
    launched 10 times on internally numbered vectors, then a plain 256 MiB device copy
    10 times: the copy's counter reading per byte calibrates the HBM traffic counters."""
    import torch
    mesh = mg.hex_mesh(32, 0.15, config=1, seed_k=6)
    space = mg.hex_space(mesh, 6, ncomp=3, config=1)
    op = mf.Operator(mf.Space.from_meshgen(space), mf.LAPLACIAN, mf.F64)
    x = torch.tensor(mg.uniform(space.ndofs, -1, 1, 1, mg.PURPOSE_X, 6), device="cuda")
    y = torch.empty_like(x)
    for _ in range(10):
        op.apply_internal(x, y)
    a = torch.ones(32 << 20, dtype=torch.float64, device="cuda")  # 256 MiB
    b = torch.empty_like(a)
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"profiled": "laplacian3-Q6 fp64 x10, copy 256MiB x10", "flops_per_apply": op.info["flops_per_apply"],
                      "bytes_per_apply": op.info["bytes_per_apply"],
                      "cell_launches_per_apply": op.info["cell_launches"]}))


def profile_q1(mf, mg):
    """The low-order kernel of the weak-scaled figures (FP64 Helmholtz, Q1, 128^3, patch
    scatter) launched 10 times, then the same 256 MiB calibration copy 10 times."""
    import torch
    mesh = mg.hex_mesh(128, 0.15, config=1, seed_k=1)
    space = mg.hex_space(mesh, 1, ncomp=1, config=1)
    op = mf.Operator(mf.Space.from_meshgen(space), mf.HELMHOLTZ, mf.F64)
    x = torch.tensor(mg.uniform(space.ndofs, -1, 1, 1, mg.PURPOSE_X, 1), device="cuda")
    y = torch.empty_like(x)
    for _ in range(10):
        op.apply_internal(x, y)
    a = torch.ones(32 << 20, dtype=torch.float64, device="cuda")  # 256 MiB
    b = torch.empty_like(a)
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"profiled": "helmholtz-Q1 128^3 fp64 x10, copy 256MiB x10",
                      "flops_per_apply": op.info["flops_per_apply"], "bytes_per_apply": op.info["bytes_per_apply"],
                      "cell_launches_per_apply": op.info["cell_launches"]}))


def profile_simplex(mf, mg):
    """The matrix-core simplex kernels for counter runs: vector P2 elasticity (48^3 x 6
    tets, patch scatter) and scalar P3 Helmholtz on the same mesh, FP64, each applied 10
    times on internally numbered vectors, then the 256 MiB calibration copy 10 times."""
    import torch
    mesh = mg.tet_mesh(48, 0.2, config=2)
    info = {}
    for k, nc, kind, name in ((2, 3, mf.ELASTICITY, "elasticity-P2"), (3, 1, mf.HELMHOLTZ, "helmholtz-P3")):
        space = mg.tet_space(mesh, k, ncomp=nc, config=2)
        op = mf.Operator(mf.Space.from_meshgen(space), kind, mf.F64, lam=1.0, mu=0.5)
        x = torch.tensor(mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_X, k), device="cuda")
        y = torch.empty_like(x)
        for _ in range(10):
            op.apply_internal(x, y)
        torch.cuda.synchronize()
        info[name] = {"flops_per_apply": op.info["flops_per_apply"], "bytes_per_apply": op.info["bytes_per_apply"],
                      "scatter": op.info["scatter"]}
        del op, x, y
    a = torch.ones(32 << 20, dtype=torch.float64, device="cuda")  # 256 MiB
    b = torch.empty_like(a)
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"profiled": "tet elasticity P2 and Helmholtz P3 48^3x6 fp64 x10 each, copy 256MiB x10"} | info))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="degrees 1..3 only (debugging)")
    ap.add_argument("--no-c4", action="store_true", help="skip the batched 64-system solves")
    ap.add_argument("--no-c5", action="store_true", help="skip the learned-preconditioner comparison")
    ap.add_argument("--c5-only", action="store_true", help="only the learned-preconditioner comparison")
    ap.add_argument("--detail-out", default=None, help="also write the detailed results (JSON) to this file")
    ap.add_argument("--c5-m", type=int, default=64, help="cells per direction of that problem")
    ap.add_argument("--simplex-only", action="store_true", help="only the simplex operator timings")
    ap.add_argument("--c4-only", action="store_true", help="only the batched 64-system solves")
    ap.add_argument("--table2", action="store_true",
                    help="only the D / Q / arithmetic-intensity table beside the paper's Table 2")
    ap.add_argument("--profile-kernel", action="store_true",
                    help="only run the dominant action kernel 10 times and a 256 MiB reference copy "
                         "(for hardware-counter runs)")
    ap.add_argument("--profile-simplex", action="store_true",
                    help="only run the tet elasticity P2 and Helmholtz P3 matrix-core kernels 10 times each "
                         "and the reference copy (for hardware-counter runs)")
    ap.add_argument("--profile-q1", action="store_true",
                    help="only run the Q1 patch kernel on 128^3 10 times and the reference copy "
                         "(for hardware-counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU design "
              "is described but not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1903_08243_amd as mf
    from paper_1903_08243_amd import meshgen as mg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    mf.load_library()
    if args.profile_kernel:
        profile_kernel(mf, mg)
        return
    if args.profile_q1:
        profile_q1(mf, mg)
        return
    if args.profile_simplex:
        profile_simplex(mf, mg)
        return
    if args.c5_only:
        print(json.dumps(bench_c5(mf, mg, m=args.c5_m)))
        return
    if args.c4_only:
        print(json.dumps({"c4": bench_c4(mf, mg), "c4_small": bench_c4(mf, mg, seed=1, m_lo=4, m_hi=12)}))
        return
    if args.simplex_only:
        print(json.dumps(bench_simplex(mf, mg)))
        return
    if args.table2:
        for row in table2(mf, mg):
            log(json.dumps(row))
        return
    degrees = [1, 2, 3] if args.quick else [1, 2, 3, 4, 5, 6]
    kinds = [("helmholtz", mf.HELMHOLTZ, 1), ("laplacian3", mf.LAPLACIAN, 3), ("laplacian1", mf.LAPLACIAN, 1)]
    log("building headline operators ...")
    cases = build_c2_cases(mf, mg, degrees, kinds)

    def step():
        for ent in cases:
            op, x, y = ent["ops"][mf.F64]
            op.apply(x, y)

    def step_internal():
        for ent in cases:
            op, x, y = ent["ops"][mf.F64]
            op.apply_internal(x, y)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(s)
        for _ in range(args.steps):
            fn()
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / args.steps, time.perf_counter() - t0

    dofs_per_step = sum(ent["ndofs"] for ent in cases)
    # headline: vectors in the workload's (random) user numbering
    t_step, wall = timed(step)
    value = dofs_per_step / t_step / 1e9
    log(f"timed {args.steps} steps (user numbering): {t_step * 1e3:.3f} ms/step, {value:.1f} GDoF/s "
        f"(wall {wall:.2f} s)")
    t_int, _ = timed(step_internal)
    value_int = dofs_per_step / t_int / 1e9
    log(f"timed {args.steps} steps (internal numbering): {t_int * 1e3:.3f} ms/step, {value_int:.1f} GDoF/s")

    # per-operator kernel timings (HIP events on the launch stream); FP64 also with cold
    # caches (a 512 MiB write before each apply)
    per = []
    flush = torch.empty(64 << 20, dtype=torch.float64, device="cuda")
    for ent in cases:
        row = {"name": ent["name"], "ndofs": ent["ndofs"]}
        for prec, tag in ((mf.F64, "fp64"), (mf.F32, "fp32")):
            op, x, y = ent["ops"][prec]
            runs = [time_kernel(op, x, y, reps=20) for _ in range(5)]  # 5 runs of 20 applies
            t = float(np.mean(runs))
            r = roof(op, t, prec)
            row[tag] = {"us": t * 1e6, "us_min": min(runs) * 1e6, "us_median": float(np.median(runs)) * 1e6,
                        "gdofs": ent["ndofs"] / t / 1e9, "frac": r["frac"], "bound": r["bound"],
                        "tflops": r["tflops"], "gbs": r["gbs"]}
            if prec == mf.F64:
                row[tag]["us_cold"] = time_kernel_cold(op, x, y, flush) * 1e6
        per.append(row)
        log(f"  {ent['name']:16s} fp64 {row['fp64']['us']:8.1f} us (cold {row['fp64']['us_cold']:8.1f}) "
            f"{row['fp64']['gdofs']:6.1f} GDoF/s roof {row['fp64']['frac']:.2f} ({row['fp64']['bound']}) | "
            f"fp32 {row['fp32']['us']:8.1f} us {row['fp32']['gdofs']:6.1f} GDoF/s roof {row['fp32']['frac']:.2f}")
    del flush
    # dominant kernel: the longest FP64 action of the step
    dom_i = int(np.argmax([p["fp64"]["us"] for p in per]))
    dom = cases[dom_i]
    op, x, y = dom["ops"][mf.F64]
    t_dom = per[dom_i]["fp64"]["us"] * 1e-6
    nl = op.info["cell_launches"]  # equal-size colour launches share the action's work evenly
    r = roof(op, t_dom, 0)
    if op.info["scatter"] == mf.SCATTER_PATCH:
        # one patch launch per apply plus the (small) sum over the nodes patches share;
        # the roofline counts the apply's work over both launches' time
        kname = (f"hex_patch_kernel<double,{dom['k'] + 1},{dom['kind']}> + simplex_shared_reduce_kernel<double> "
                 f"({dom['name']})")
    else:
        kname = f"hex_apply_kernel<double,{dom['k'] + 1},{dom['kind']}> ({dom['name']})"
    traffic = measured_traffic() if (dom["k"], dom["kind"], dom["ncomp"]) == (6, mf.LAPLACIAN, 3) else None
    if r["bound"] == "alu":
        roofline = {"bound": "alu", "achieved": r["flops"] / t_dom / 1e12, "peak": PEAK_FP64 / 1e12,
                    "unit": "TFLOP/s", "frac": r["flops"] / t_dom / PEAK_FP64, "traffic": traffic,
                    "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                    "kernel": kname,
                    "flops_per_launch": r["flops"] / nl, "bytes_per_launch": r["bytes"] / nl,
                    "launch_us": t_dom * 1e6 / nl, "launches_per_apply": nl}
    else:
        roofline = {"bound": "hbm", "achieved": r["bytes"] / t_dom / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                    "frac": r["bytes"] / t_dom / PEAK_HBM, "traffic": traffic,
                    "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                    "kernel": kname,
                    "flops_per_launch": r["flops"] / nl, "bytes_per_launch": r["bytes"] / nl,
                    "launch_us": t_dom * 1e6 / nl, "launches_per_apply": nl}

    extra = {}
    try:
        extra["simplex"] = bench_simplex(mf, mg)
    except Exception as ex:  # reported, never silently replaced
        extra["simplex"] = {"error": repr(ex)}
    if not args.quick:
        try:
            extra["hex_weak_scaled"] = bench_weak(mf, mg)
        except Exception as ex:
            extra["hex_weak_scaled"] = {"error": repr(ex)}
    try:
        extra["hex_q_k+2"] = bench_hex_q(mf, cases)
    except Exception as ex:  # reported, never silently replaced
        extra["hex_q_k+2"] = {"error": repr(ex)}
    try:
        extra["table2"] = table2(mf, mg)
    except Exception as ex:  # reported, never silently replaced
        extra["table2"] = {"error": repr(ex)}
    try:
        extra["cg"] = bench_cg(mf, mg)
        log(f"  cg: {json.dumps(extra['cg'])}")
    except Exception as ex:  # reported, never silently replaced
        extra["cg"] = {"error": repr(ex)}
    cpu, parity = None, None
    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample ...")
        cpu, parity = cpu_baseline(mg, cases)
        log(f"  cpu oracle: {cpu['value']:.4f} GDoF/s on {cpu['cores']} threads; GPU against it: "
            f"{parity['max_rel_error_fp64']:.2e} (fp64), {parity['max_rel_error_fp32']:.2e} (fp32)")
    n_ops = len(cases)
    if not args.quick and not args.no_c4:
        del cases  # free the headline operators before the batched workload
        torch.cuda.empty_cache()
        try:
            log("batched solves (64 Helmholtz systems) ...")
            extra["c4_batched"] = bench_c4(mf, mg)
            log(f"  c4: {json.dumps({k: v for k, v in extra['c4_batched'].items() if k not in ('mesh_m', 'degree')})}")
        except Exception as ex:
            extra["c4_batched"] = {"error": repr(ex)}
        try:
            log("batched solves (64 small Helmholtz systems, 4^3..12^3 cells) ...")
            extra["c4_batched_small"] = bench_c4(mf, mg, seed=1, m_lo=4, m_hi=12)
            log(f"  c4 small: {json.dumps({k: v for k, v in extra['c4_batched_small'].items() if k not in ('mesh_m', 'degree')})}")
        except Exception as ex:
            extra["c4_batched_small"] = {"error": repr(ex)}
    if not args.quick and not args.no_c5:
        torch.cuda.empty_cache()
        try:
            log("learned preconditioner (variable-kappa Poisson Q3 64^3) ...")
            extra["c5_learned_precond"] = bench_c5(mf, mg)
        except Exception as ex:
            extra["c5_learned_precond"] = {"error": repr(ex)}

    peaks = None
    try:
        peaks = mf.probe_peaks()
        log(f"  attainable peaks: {json.dumps(peaks)}")
    except Exception as ex:  # reported, never silently replaced
        peaks = {"error": repr(ex)}
    if isinstance(roofline, dict) and isinstance(peaks, dict) and "error" not in peaks:
        att = peaks["fp64_vector_tflops"] if roofline["bound"] == "alu" else peaks["hbm_copy_gbs"]
        roofline["attainable_peak"] = att
        roofline["frac_of_attainable"] = roofline["achieved"] / att

    detail = {
        "config": {"cells": 32768, "degrees": degrees, "operators_per_step": n_ops,
                   "dofs_per_step": dofs_per_step},
        "internal_numbering": {"value": value_int, "unit": "GDoF/s", "ms_per_step": t_int * 1e3,
                               "note": "same step with vectors in the library's cell-order node numbering "
                                       "(no boundary permutation), as used inside CG"},
        "measured_peaks": peaks, "roofline": roofline, "cpu_baseline": cpu, "parity_vs_oracle": parity,
        "per_operator": per, **extra,
    }
    log("detail " + json.dumps(detail))
    if args.detail_out:
        with open(args.detail_out, "w") as f:
            json.dump(detail, f, indent=1)
    # the one line the harness reads: compact, under 2 KB
    rl = None
    if isinstance(roofline, dict):
        rl = {k: roofline[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")}
        rl["kernel"] = roofline["kernel"]
        if "attainable_peak" in roofline:
            rl["attainable_peak"] = round(roofline["attainable_peak"], 2)
    par = None
    if parity:
        par = {"fp64": parity["max_rel_error_fp64"], "fp32": parity["max_rel_error_fp32"],
               "tol_fp64": 1e-12, "tol_fp32": 1e-5, "operators": parity["operators"]}
    cpu_c = None
    if cpu:
        cpu_c = {k: cpu[k] for k in ("value", "unit", "cores", "kind")}
        cpu_c["sample"] = cpu["sample"][:160]
    out = {
        "metric": METRIC, "value": value, "unit": "GDoF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_step * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "FP64 Helmholtz + Laplacian (ncomp 3, 1) actions, Q1..Q6 GLL, (k+1)^3 Gauss, "
                               "32^3 hex perturbed +-0.15h, random renumbering",
                   "operators_per_step": n_ops, "dofs_per_step": dofs_per_step},
        "roofline": rl, "cpu_baseline": cpu_c, "parity_vs_oracle": par,
    }
    line = json.dumps(out)
    assert len(line) < 2048, f"summary line is {len(line)} bytes"
    print(line, flush=True)


if __name__ == "__main__":
    main()
