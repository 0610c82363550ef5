"""Benchmark of the matrix-free phase-field operator on one MI355X.

One step = one pass of the hot path over the workload: FP64 residual apply,
FP64 Jacobian apply, FP64 adjoint apply (with parameter gradient) and, when the
multigrid is built, the FP32 linearised apply and one FP32 p-multigrid V-cycle.
Inputs are generated once and resident in HBM before the timed region.

value = Jacobian-apply DoFs/s (FP64) = 4 n_nodes / median Jacobian-apply time.
The headline's outputs are compared with the oracle on every node (rel-L2 and, per field,
the largest entry error over the largest reference entry).
Beside the headline the line carries side legs on other workloads: the third
example's branches in parallel, curved (mapped) elements, a mesh given by its
element-to-node table (with a hole), the order-2 mesh and one Newton step on the Q4 box (FGMRES, and the conjugate-gradient variant beside it);
with --newton-all also Newton steps with branches and on the curved mesh.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# What the paper states about its own runs (Section 5, computing environment): no per-apply
# throughput is given, only the scale of the microstructure runs and their hardware.
PAPER_CONTEXT = {
    "per_apply_throughput": None,
    "hardware": "AMD Instinct MI250X (gfx90a), 4 per node, each run as 2 logical GPUs; 64 EPYC cores and "
                "512 GB host memory per node",
    "largest_problem_dofs_approx": 2.0e7,
    "time_steps_approx": 500,
    "logical_gpus_max": 24,
    "nodes_max": 3,
    "allocation_hours": 12,
    "derived_wall_s_per_step": 12 * 3600 / 500,
    "elements": "quadratic tetrahedra, unstructured microstructure meshes",
}
HBM_PEAK_GBS = 8000.0
FP64_VEC_PEAK_TFLOPS = 78.6
CSRC = os.path.join(ROOT, "paper_2607_21150_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_op64_q3_jacobian_C3_hbm_counters.md")


def kernel_source_digest():
    """sha256 over the HIP sources (sorted by name): identifies the kernels the counters belong to."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".hpp", ".h")):
            h.update(name.encode())
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def measured_counters(config):
    """Per-Jacobian-apply counter values from the committed summary (HBM bytes, FP64 VALU and
    matrix-core FLOPs), or {} when the summary is missing, was taken on another workload, or the
    kernel sources changed since it was taken."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if line.startswith("- ") and " = " in line:
                    k, v = line[2:].split(" = ", 1)
                    kv[k.strip().strip("`")] = v.strip().strip("`")
        if kv.get("source_sha256") != kernel_source_digest() or kv.get("config") != config:
            return {}
        return {k: float(kv[k]) for k in ("hbm_bytes_per_apply", "valu_fp64_flops_per_apply",
                                          "mfma_f64_flops_per_apply") if k in kv}
    except (OSError, KeyError, ValueError):
        return {}


def measured_traffic(config):
    """HBM bytes per Jacobian apply from the committed counter summary, or None (see measured_counters)."""
    return measured_counters(config).get("hbm_bytes_per_apply")


def copy_probe(torch, nbytes=1 << 30, reps=10):
    """Device-to-device copy of a known size: achievable HBM GB/s (read + write) on this GPU. Its
    kernel also calibrates the FETCH_SIZE / WRITE_SIZE counters."""
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    return {"bytes_per_copy": 2 * nbytes, "ms": t * 1e3, "gbs": 2 * nbytes / t / 1e9}


def alg_bytes(mesh, kind):
    """Minimal algorithmic HBM bytes of one apply: every nodal value read or written once,
    the per-point state (8 doubles) and phase id (1 byte) read once."""
    nodes, qps = mesh.n_nodes, mesh.n_q
    if kind == "residual":      # z (4) + phi_n (1) read, r (4) written
        return 72 * nodes + 65 * qps
    if kind in ("jacobian", "adjoint"):  # z, dz read, y written
        return 96 * nodes + 65 * qps
    if kind == "fp32_apply":    # design C: FP32 z, dz, y (48 B per node); 46 B record per point
        return 48 * nodes + 46 * qps
    if kind == "jacobian_stored":  # the same operator as the recompute Jacobian: priced on its bytes
        return 96 * nodes + 65 * qps
    raise ValueError(kind)


def stored_bytes(mesh, kind):
    """Bytes the record applies actually read and write (larger than the algorithmic bytes,
    which do not grow with what is stored): FP32 apply: u mirror (12), dz (16), y (16) per
    node, record 60 + flags 1 + phase 1 per point; stored FP64 Jacobian: u copy (24), dz (32),
    y (32) per node, record 120 + flags 1 + phase 1 per point."""
    if kind == "fp32_apply":
        return 44 * mesh.n_nodes + 62 * mesh.n_q
    if kind == "jacobian_stored":
        return 88 * mesh.n_nodes + 122 * mesh.n_q
    raise ValueError(kind)


def whole_mesh_err(gpu_vec, ref):
    """Error of a [4][n_nodes] GPU result against the oracle on every node: rel-L2 and, per
    field, max |gpu - ref| / max |ref| (the largest over the four fields)."""
    gpu_vec = np.asarray(gpu_vec, dtype=np.float64)
    rel = float(np.linalg.norm(gpu_vec - ref) / max(np.linalg.norm(ref), 1e-300))
    worst = 0.0
    for f in range(ref.shape[0]):
        s = float(np.max(np.abs(ref[f])))
        if s > 0.0:
            worst = max(worst, float(np.max(np.abs(gpu_vec[f] - ref[f]))) / s)
    return {"rel_l2": rel, "max_entry": worst}


def cpu_baseline(d, seconds=10.0):
    """The oracle (as it stands) on the host cores, on a bounded sample of elements."""
    from oracle import pyoracle
    pyoracle.build(force=False)
    orc = pyoracle.Oracle.from_inputs(d)
    mesh = d["mesh"]
    # calibrate on a small sample, then size the timed sample to ~`seconds`
    n_cal = min(mesh.n_elem, 256)
    t0 = time.perf_counter()
    orc.jacobian(d["z"], d["dz"], elems=np.arange(n_cal, dtype=np.int32), check=False)
    t_cal = max(time.perf_counter() - t0, 1e-4)
    n = int(min(mesh.n_elem, max(n_cal, n_cal * seconds / t_cal)))
    elems = np.arange(n, dtype=np.int32)
    t0 = time.perf_counter()
    orc.jacobian(d["z"], d["dz"], elems=elems, check=False)
    t = time.perf_counter() - t0
    frac = n / mesh.n_elem
    dofs_per_s = mesh.n_dof / (t / frac)
    cores = pyoracle.num_threads()
    # the same on one core, on a sample of 1/cores of the elements
    n1 = max(1, n // max(cores, 1))
    pyoracle.set_num_threads(1)
    t0 = time.perf_counter()
    orc.jacobian(d["z"], d["dz"], elems=np.arange(n1, dtype=np.int32), check=False)
    t1 = time.perf_counter() - t0
    pyoracle.set_num_threads(cores)
    model = cpu_description()
    return {"value": dofs_per_s, "unit": "DoF/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 Jacobian apply on elements 0..{n - 1} ({n} of {mesh.n_elem}, {frac:.3f} of the work) "
                      f"took {t:.2f} s on {cores} threads; scaled to the full apply",
            "value_1core": mesh.n_dof / (t1 * mesh.n_elem / n1),
            "sample_1core": f"elements 0..{n1 - 1} on 1 thread took {t1:.2f} s",
            "cpu_model": model, "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS")}


def cpu_description():
    """Host CPU as /proc/cpuinfo names it (model name, family/model/stepping, sockets, cores
    per socket) and the CPUs this process may run on."""
    info, sockets, cores = {}, set(), {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" not in line:
                    continue
                k, v = (x.strip() for x in line.split(":", 1))
                if k in ("model name", "cpu family", "model", "stepping", "cpu MHz") and k not in info:
                    info[k] = v
                if k == "physical id":
                    sockets.add(v)
                if k == "cpu cores":
                    cores[len(sockets)] = v
    except OSError:
        return "unknown"
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count()
    return (f"{info.get('model name', 'unknown')} (family {info.get('cpu family', '?')}, model "
            f"{info.get('model', '?')}, stepping {info.get('stepping', '?')}, {info.get('cpu MHz', '?')} MHz; "
            f"{len(sockets) or '?'} socket(s), {next(iter(cores.values()), '?')} cores per socket; "
            f"{os.cpu_count()} logical CPUs, {avail} available to this process)")


def secondary_leg(torch, I, pfmf, config):
    """Device time of each apply on a second workload (mean of 20 back-to-back applies after
    3 warm-up ones): the Q2 counterpart of the headline Q3 configuration."""
    d = I.make_inputs(config, "base")
    mesh = d["mesh"]
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", torch.float64)
    ctx = pfmf.Context.from_inputs(d)
    z, dz, v = dev(d["z"]), dev(d["dz"]), dev(d["v_top"])
    y, g = torch.empty_like(z), torch.empty_like(z)
    gp = torch.empty((len(d["phases"]), 3), dtype=torch.float64, device="cuda")
    ctx.linearize(z)
    dz32 = dz.float()
    y32 = torch.empty_like(dz32)
    ms = {}
    for name, f in (("residual", lambda: ctx.apply_residual(z, y)),
                    ("jacobian", lambda: ctx.apply_jacobian(z, dz, y)),
                    ("adjoint", lambda: ctx.apply_adjoint(z, v, g, gp)),
                    ("fp32_apply", lambda: ctx.apply_jacobian_f32(0, dz32, y32)),
                    ("jacobian_stored", lambda: ctx.apply_jacobian_lin(dz, g))):
        for _ in range(3):
            f()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(20):
            f()
        b.record()
        torch.cuda.synchronize()
        ms[name] = a.elapsed_time(b) / 20
    ctx.check()
    return {"config": f"{config} Q{mesh.p} {mesh.nx}^3, {mesh.n_dof} DoFs", "ms": ms,
            "dofs_per_s": {k: mesh.n_dof / (t * 1e-3) for k, t in ms.items()},
            "gbs_alg": {k: alg_bytes(mesh, k) / (t * 1e-3) / 1e9 for k, t in ms.items()},
            "hbm_frac_alg": {k: alg_bytes(mesh, k) / (t * 1e-3) / 1e9 / HBM_PEAK_GBS for k, t in ms.items()},
            "fp32_over_fp64_apply_speedup": ms["jacobian"] / ms["fp32_apply"],
            "fp32_over_stored_fp64_speedup": ms["jacobian_stored"] / ms["fp32_apply"]}


def branch_state_bytes(d):
    """Algorithmic bytes of the extra branches' state per apply: D (6 doubles) of every
    inelastic extra branch at the points of its phase, plus the accumulated plastic strain
    of a Prandtl branch (a Hooke branch reads none)."""
    total = 0
    for pid, row in enumerate(d["branches"]):
        npts = int(np.count_nonzero(d["phase"] == pid))
        for b in row:
            if b.kind == 2:
                total += 48 * npts
            elif b.kind == 3:
                total += 56 * npts
    return total


def branches_leg(torch, I, pfmf, config, steps=20, warmup=3):
    """FP64 applies with the third example's matrix (perfectly plastic Prandtl block in
    parallel with a Hooke spring and a Maxwell branch; Hooke particles) on a workload of the
    headline's size: median device time of each apply (HIP events around every launch)."""
    d = I.make_inputs(config, "ex3")
    mesh = d["mesh"]
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", torch.float64)
    ctx = pfmf.Context.from_inputs(d)
    z, dz, v = dev(d["z"]), dev(d["dz"]), dev(d["v_top"])
    r, y, g = torch.empty_like(z), torch.empty_like(z), torch.empty_like(z)
    gp = torch.empty((len(d["phases"]), 3), dtype=torch.float64, device="cuda")
    ctx.linearize(z)
    dz32 = dz.float()
    y32, b32, x32, ys = torch.empty_like(dz32), torch.empty_like(dz32), torch.empty_like(dz32), torch.empty_like(z)
    ctx.apply_jacobian_f32(0, dz32, b32)
    ops = {"vcycle": lambda: ctx.pmg_vcycle(b32, x32), "fp32_apply": lambda: ctx.apply_jacobian_f32(0, dz32, y32),
           "residual": lambda: ctx.apply_residual(z, r), "jacobian": lambda: ctx.apply_jacobian(z, dz, y),
           "adjoint": lambda: ctx.apply_adjoint(z, v, g, gp), "jacobian_stored": lambda: ctx.apply_jacobian_lin(dz, ys)}
    for _ in range(warmup):
        for f in ops.values():
            f()
    torch.cuda.synchronize()
    ev = {k: [] for k in ops}
    for _ in range(steps):
        for k, f in ops.items():
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            f()
            b.record()
            ev[k].append((a, b))
    torch.cuda.synchronize()
    ctx.check()
    ms = {k: float(np.median([a.elapsed_time(b) for a, b in ev[k]])) for k in ev}
    t0 = time.perf_counter()
    ctx.linearize(z)
    ms["linearize"] = (time.perf_counter() - t0) * 1e3  # host wall time (the call synchronises)
    xb = branch_state_bytes(d)
    n_layers = 1 + len(d["branches"][0])
    alg = {k: alg_bytes(mesh, k) + xb for k in ("residual", "jacobian", "adjoint")}
    # record applies: every layer's record is read (61 B per point and layer for FP32, 121 B
    # for the stored FP64 linearisation), on top of the block-only bytes
    alg["fp32_apply"] = alg_bytes(mesh, "fp32_apply") + 61 * (n_layers - 1) * mesh.n_q
    alg["jacobian_stored"] = alg_bytes(mesh, "jacobian_stored") + 121 * (n_layers - 1) * mesh.n_q
    errs = {}
    try:
        from oracle import pyoracle
        pyoracle.build(force=False)
        orc = pyoracle.Oracle.from_inputs(d)
        jref = orc.jacobian(d["z"], d["dz"])
        errs["jacobian"] = whole_mesh_err(y.cpu().numpy(), jref)
        errs["fp32_apply"] = whole_mesh_err(y32.double().cpu().numpy(), jref)
        errs["jacobian_stored"] = whole_mesh_err(ys.cpu().numpy(), jref)
        del jref
        errs["adjoint"] = whole_mesh_err(g.cpu().numpy(), orc.adjoint(d["z"], d["v_top"])[0])
        errs["nodes_compared"] = mesh.n_nodes
    except Exception as exc:
        errs["error"] = str(exc)
    return {"config": f"{config} Q{mesh.p} {mesh.nx}^3, {mesh.n_dof} DoFs, matrix = perfectly plastic Prandtl "
                      f"|| Hooke || Maxwell, particle = Hooke (particle fraction {d['vol_frac']:.3f}, e0={d['e0']})",
            "ms_median": ms, "dofs_per_s": {k: mesh.n_dof / (ms[k] * 1e-3) for k in alg},
            "alg_bytes_per_apply": alg,
            "gbs_alg": {k: alg[k] / (ms[k] * 1e-3) / 1e9 for k in alg},
            "fp32_over_fp64_apply_speedup": ms["jacobian"] / ms["fp32_apply"],
            "rel_err_vs_oracle": errs}


def geometry_leg(torch, I, pfmf, config, steps=20, warmup=3, with_box=False):
    """Applies on mapped (curved) Q3 elements: the headline's plastic workload with its node
    lattice moved by a smooth bump of 0.2 h, the per-point J^-1 and weight read from the
    stored geometry record (80 B per point on top of the box's bytes): the FP64 residual,
    Jacobian and adjoint, and the FP32 multigrid (linearisation, fine apply, stored FP64
    apply, V-cycle). Median device time of each (HIP events around every launch); with_box:
    the same on the box mesh too, for the ratio (they launch the headline's kernels on other
    inputs, so a profiled run leaves them out)."""
    d = I.make_inputs(config, "plastic", geometry="curved")
    mesh = d["mesh"]
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", torch.float64)
    ctx = pfmf.Context.from_inputs(d)
    z, dz, v = dev(d["z"]), dev(d["dz"]), dev(d["v_top"])
    r, y, g = torch.empty_like(z), torch.empty_like(z), torch.empty_like(z)
    gp = torch.empty((len(d["phases"]), 3), dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    ctx.set_geometry(dev(d["X"]))
    setup_ms = (time.perf_counter() - t0) * 1e3  # host wall time of the setup call (it synchronises)
    ops = {"residual": lambda: ctx.apply_residual(z, r), "jacobian": lambda: ctx.apply_jacobian(z, dz, y),
           "adjoint": lambda: ctx.apply_adjoint(z, v, g, gp)}
    # the FP32 multigrid on the same mesh: linearisation, fine apply, stored FP64 apply, V-cycle
    t0 = time.perf_counter()
    ctx.linearize(z)
    lin_ms = (time.perf_counter() - t0) * 1e3  # host wall time (the call synchronises)
    dz32 = dz.float()
    y32, b32, x32, ys = torch.empty_like(dz32), torch.empty_like(dz32), torch.empty_like(dz32), torch.empty_like(z)
    ctx.apply_jacobian_f32(0, dz32, b32)
    ops.update({"fp32_apply": lambda: ctx.apply_jacobian_f32(0, dz32, y32),
                "jacobian_stored": lambda: ctx.apply_jacobian_lin(dz, ys), "vcycle": lambda: ctx.pmg_vcycle(b32, x32)})

    def timed():
        for _ in range(warmup):
            for f in ops.values():
                f()
        torch.cuda.synchronize()
        ev = {k: [] for k in ops}
        for _ in range(steps):
            for k, f in ops.items():
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                f()
                b.record()
                ev[k].append((a, b))
        torch.cuda.synchronize()
        ctx.check()
        return {k: float(np.median([a.elapsed_time(b) for a, b in ev[k]])) for k in ev}

    ms = timed()
    ms["linearize"] = lin_ms
    y_cur, g_cur, y32_cur = y.cpu().numpy(), g.cpu().numpy(), y32.double().cpu().numpy()
    ms_box = None
    if with_box:
        ctx.set_geometry(None)
        ctx.linearize(z)
        ms_box = timed()
    # algorithmic bytes: the box's plus the geometry record (80 B per point in FP64, 40 B in
    # the FP32 copy the FP32 levels read) for the applies that read it (the V-cycle is timed only)
    alg = {k: alg_bytes(mesh, k) + (40 if k == "fp32_apply" else 80) * mesh.n_q for k in ops if k != "vcycle"}
    errs = {}
    try:
        from oracle import pyoracle
        pyoracle.build(force=False)
        orc = pyoracle.Oracle.from_inputs(d)
        jref = orc.jacobian(d["z"], d["dz"])
        errs["jacobian"] = whole_mesh_err(y_cur, jref)
        errs["fp32_apply"] = whole_mesh_err(y32_cur, jref)
        del jref
        errs["adjoint"] = whole_mesh_err(g_cur, orc.adjoint(d["z"], d["v_top"])[0])
        errs["nodes_compared"] = mesh.n_nodes
    except Exception as exc:
        errs["error"] = str(exc)
    return {"config": f"{config} Q{mesh.p} {mesh.nx}^3 curved (bump 0.2 h), {mesh.n_dof} DoFs, plastic matrix",
            "ms_median": ms, "setup_ms": setup_ms,
            "dofs_per_s": {k: mesh.n_dof / (ms[k] * 1e-3) for k in alg},
            "alg_bytes_per_apply": alg,
            "gbs_alg": {k: alg[k] / (ms[k] * 1e-3) / 1e9 for k in alg},
            "fp32_over_fp64_apply_speedup": ms["jacobian"] / ms["fp32_apply"],
            **({"ms_median_box": ms_box, "curved_over_box_time": {k: ms[k] / ms_box[k] for k in ms_box}}
               if ms_box else {}),
            "rel_err_vs_oracle": errs}


def table_leg(torch, I, pfmf, config, steps=20, warmup=3, hole=0.15):
    """FP64 applies on a mesh given by its element-to-node table (pf_setup_mesh_table): the
    headline's plastic workload with the elements inside a cylindrical hole of radius `hole`
    mm removed, every element in one of the 24 cube orientations, elements in lattice order
    and nodes numbered by first touch. Median device time of each apply (HIP events around
    every launch) and whole-mesh errors against the oracle. Algorithmic bytes add the
    geometry record (80 B per point) and the table (4 B per element node) to the box's."""
    t_gen = time.perf_counter()
    d = I.unstructured(I.make_inputs(config, "plastic"), hole_radius=hole, node_order="first_touch",
                       shuffle_elements=False)
    mesh = d["mesh"]
    print(f"[bench] table inputs {config}: {mesh.n_elem} elements, {mesh.n_dof} DoFs, generated in "
          f"{time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", torch.float64)
    t0 = time.perf_counter()
    ctx = pfmf.Context.from_inputs(d)
    setup_ms = (time.perf_counter() - t0) * 1e3  # host wall time: table copy, CSR map, geometry record
    z, dz, v = dev(d["z"]), dev(d["dz"]), dev(d["v_rand"])
    r, y, g = torch.empty_like(z), torch.empty_like(z), torch.empty_like(z)
    gp = torch.empty((len(d["phases"]), 3), dtype=torch.float64, device="cuda")
    ops = {"residual": lambda: ctx.apply_residual(z, r), "jacobian": lambda: ctx.apply_jacobian(z, dz, y),
           "adjoint": lambda: ctx.apply_adjoint(z, v, g, gp)}
    for _ in range(warmup):
        for f in ops.values():
            f()
    torch.cuda.synchronize()
    ev = {k: [] for k in ops}
    for _ in range(steps):
        for k, f in ops.items():
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            f()
            b.record()
            ev[k].append((a, b))
    torch.cuda.synchronize()
    ctx.check()
    ms = {k: float(np.median([a.elapsed_time(b) for a, b in ev[k]])) for k in ev}
    rr, yy, gg = r.cpu().numpy(), y.cpu().numpy(), g.cpu().numpy()
    del ctx, z, dz, v, r, y, g
    torch.cuda.empty_cache()
    P3 = (mesh.p + 1) ** 3
    extra = 80 * mesh.n_q + 4 * P3 * mesh.n_elem
    alg = {"residual": 72 * mesh.n_nodes + 65 * mesh.n_q + extra,
           "jacobian": 96 * mesh.n_nodes + 65 * mesh.n_q + extra,
           "adjoint": 96 * mesh.n_nodes + 65 * mesh.n_q + extra}
    errs = {}
    try:
        from oracle import pyoracle
        pyoracle.build(force=False)
        orc = pyoracle.Oracle.from_inputs(d)
        errs["residual"] = whole_mesh_err(rr, orc.residual(d["z"]))
        errs["jacobian"] = whole_mesh_err(yy, orc.jacobian(d["z"], d["dz"]))
        errs["adjoint"] = whole_mesh_err(gg, orc.adjoint(d["z"], d["v_rand"])[0])
        errs["nodes_compared"] = mesh.n_nodes
    except Exception as exc:
        errs["error"] = str(exc)
    return {"config": f"{config} Q{mesh.p}, {mesh.n_elem} elements of the {mesh.box.nx}^3 lattice (cylindrical hole "
                      f"of radius {hole} mm), each in one of the 24 cube orientations, nodes numbered by first "
                      f"touch; {mesh.n_dof} DoFs, plastic matrix",
            "ms_median": ms, "setup_ms": setup_ms,
            "dofs_per_s": {k: mesh.n_dof / (ms[k] * 1e-3) for k in ms},
            "alg_bytes_per_apply": alg,
            "gbs_alg": {k: alg[k] / (ms[k] * 1e-3) / 1e9 for k in ms},
            "hbm_frac_alg": {k: alg[k] / (ms[k] * 1e-3) / 1e9 / HBM_PEAK_GBS for k in ms},
            "rel_err_vs_oracle": errs}


def newton_leg(torch, I, pfmf, config, variant="base", cheb_degree=3, coarse_sweeps=32, restart=30,
               geometry="box", with_cg=False, h_levels=False, h_coarse_sweeps=8):
    """One Newton step on a uniaxial-tension box: u_x = 0 on x = 0, u_y = 0 on y = 0, u_z = 0 on
    z = 0, u_z = e0 lz on z = lz; FGMRES(30) to 1e-8 with one FP32 V-cycle per iteration
    (levels p -> 2 -> 1 for p = 4, else p -> ... -> 1; Chebyshev(3); 32 sweeps on the order-1
    level, assembled as a block stencil), FP64 Jacobian as the operator. h_levels: below the
    order-1 level the hierarchy continues on order-1 lattices halved per direction while the
    element counts stay even (Galerkin stencils), with h_coarse_sweeps sweeps on the coarsest;
    the step with the p-levels alone is then reported beside it. geometry="curved": the same
    on the curved mesh (planar boundary faces, so the same faces are constrained).
    with_cg: the same step again from the same start with preconditioned conjugate gradients
    (the same V-cycle, at most 300 iterations), its outcome reported beside FGMRES."""
    t_gen = time.perf_counter()
    d = I.make_inputs(config, variant, geometry=geometry)
    mesh = d["mesh"]
    print(f"[bench] newton inputs {config}/{variant}: {mesh.n_dof} DoFs, generated in {time.perf_counter() - t_gen:.1f} s",
          file=sys.stderr, flush=True)
    nx1, ny1, nz1 = mesh.node_dims
    i = np.arange(mesh.n_nodes)
    ix, iy, iz = i % nx1, (i // nx1) % ny1, i // (nx1 * ny1)
    z0 = d["z"].copy()
    z0[0, ix == 0] = 0.0
    z0[1, iy == 0] = 0.0
    z0[2, iz == 0] = 0.0
    z0[2, iz == nz1 - 1] = d["e0"] * mesh.lz
    ctx = pfmf.Context.from_inputs(d)
    p_levels = [4, 2, 1] if mesh.p == 4 else list(range(mesh.p, 0, -1))
    levels = list(p_levels)
    p_sweeps = coarse_sweeps
    if h_levels:
        ne = [mesh.nx, mesh.ny, mesh.nz]
        while len(levels) < 8 and all(n % 2 == 0 and n >= 2 for n in ne):
            levels.append(1)
            ne = [n // 2 for n in ne]
        coarse_sweeps = h_coarse_sweeps
    ctx.set_pmg_levels(levels)
    ctx.set_dirichlet({"x0": ["ux"], "y0": ["uy"], "z0": ["uz"], "z1": ["uz"]})
    z = torch.as_tensor(z0).to("cuda", torch.float64)
    dz = torch.as_tensor(np.ascontiguousarray(d["dz"])).to("cuda", torch.float64)
    # FP64 and FP32 fine applies on this workload (device time of 10 back-to-back applies)
    ctx.linearize(z)
    y = torch.empty_like(z)
    dz32 = dz.float()
    y32 = torch.empty_like(dz32)
    ms = {}
    ys = torch.empty_like(z)
    for name, f in (("jacobian", lambda: ctx.apply_jacobian(z, dz, y)),
                    ("jacobian_stored", lambda: ctx.apply_jacobian_lin(dz, ys)),
                    ("fp32_apply", lambda: ctx.apply_jacobian_f32(0, dz32, y32)),
                    ("vcycle", lambda: ctx.pmg_vcycle(dz32, y32))):
        f()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(10):
            f()
        b.record()
        torch.cuda.synchronize()
        ms[name] = a.elapsed_time(b) / 10
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = ctx.newton_step(z, rtol=1e-8, restart=restart, max_iters=300, cheb_degree=cheb_degree,
                          coarse_sweeps=coarse_sweeps, raise_on_noconv=False)
    t_step = time.perf_counter() - t0
    print(f"[bench] newton step {rep} in {t_step:.2f} s", file=sys.stderr, flush=True)
    out = {"config": f"{config} Q{mesh.p} {mesh.nx}^3, {mesh.n_dof} DoFs, uniaxial faces, levels {levels}"
                     + (f", materials '{variant}'" if variant != "base" else "")
                     + (", curved elements (bump 0.2 h)" if geometry != "box" else "")
                     + f", FGMRES({restart}), Chebyshev({cheb_degree}), {coarse_sweeps} coarse sweeps",
           "time_to_solution_s": t_step, "fgmres_iterations": rep["iterations"],
           "gram_schmidt_refinements": rep["refinements"],
           "converged": bool(rep["converged"]), "rel_res_true": rep["res_true"] / max(rep["res0"], 1e-300),
           "t_linearize_ms": rep["t_linearize_ms"], "ms": ms,
           "dofs_per_s": {k: mesh.n_dof / (ms[k] * 1e-3) for k in ("jacobian", "jacobian_stored", "fp32_apply")},
           "fp32_over_fp64_apply_speedup": ms["jacobian"] / ms["fp32_apply"],
           "fp32_over_stored_fp64_speedup": ms["jacobian_stored"] / ms["fp32_apply"]}
    if levels != p_levels:
        # the same step with the p-levels alone (coarse_sweeps Chebyshev sweeps on the order-1 stencil)
        ctx.set_pmg_levels(p_levels)
        zp = torch.as_tensor(z0).to("cuda", torch.float64)
        ctx.linearize(zp)  # allocates the hierarchy outside the timed step
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rp = ctx.newton_step(zp, rtol=1e-8, restart=restart, max_iters=300, cheb_degree=cheb_degree,
                             coarse_sweeps=p_sweeps, raise_on_noconv=False)
        t_p = time.perf_counter() - t0
        print(f"[bench] newton step, p-levels {p_levels} only: {rp} in {t_p:.2f} s", file=sys.stderr, flush=True)
        out["p_levels_only"] = {"levels": p_levels, "coarse_sweeps": p_sweeps, "time_to_solution_s": t_p,
                                "fgmres_iterations": rp["iterations"], "converged": bool(rp["converged"]),
                                "rel_res_true": rp["res_true"] / max(rp["res0"], 1e-300)}
        ctx.set_pmg_levels(levels)
        ctx.linearize(zp)
    if with_cg:
        zc = torch.as_tensor(z0).to("cuda", torch.float64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cg = ctx.newton_step(zc, rtol=1e-8, restart=restart, max_iters=300, cheb_degree=cheb_degree,
                             coarse_sweeps=coarse_sweeps, raise_on_noconv=False, krylov="cg")
        t_cg = time.perf_counter() - t0
        print(f"[bench] newton step (CG) {cg} in {t_cg:.2f} s", file=sys.stderr, flush=True)
        out["cg"] = {"time_s": t_cg, "iterations": cg["iterations"], "converged": bool(cg["converged"]),
                     "breakdown": bool(cg["breakdown"]),
                     "rel_res_true": cg["res_true"] / max(cg["res0"], 1e-300),
                     "rel_res_cg": cg["res_lin"] / max(cg["res0"], 1e-300),
                     "update_rel_diff_vs_fgmres": float(torch.linalg.norm((zc - z)) /
                                                         max(float(torch.linalg.norm(z - torch.as_tensor(z0).to(
                                                             "cuda", torch.float64))), 1e-300))}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="C3")
    ap.add_argument("--variant", default="base")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-oracle", action="store_true",
                    help="skip the whole-mesh oracle comparison of the headline workload (profiled runs)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-newton", action="store_true",
                    help="skip the Newton step (FGMRES + FP32 p-MG, and the CG variant) on --newton-config")
    ap.add_argument("--newton-all", action="store_true",
                    help="also the Newton steps with the third example's branches and on the curved mesh")
    ap.add_argument("--newton-config", default="C5")
    ap.add_argument("--secondary", default="C2",
                    help="second workload whose applies are timed and reported beside the headline ('' = none)")
    ap.add_argument("--newton-branches-config", default="C2",
                    help="workload of the Newton step with the third example's branches (with --newton-all; "
                         "'' = none)")
    ap.add_argument("--branches", default="C3",
                    help="workload on which the applies with the third example's branches in parallel are timed "
                         "('' = none)")
    ap.add_argument("--geometry", default="C3",
                    help="workload on which the applies on curved (mapped) Q3 elements are timed ('' = none)")
    ap.add_argument("--newton-curved-config", default="C5",
                    help="workload of the Newton step on the curved mesh (with --newton-all; '' = none)")
    ap.add_argument("--table", default="C3",
                    help="workload on which the applies on a mesh given by its element table are timed ('' = none)")
    ap.add_argument("--geometry-box", action="store_true",
                    help="also time the geometry leg's applies on the box mesh (the curved / box ratio)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU sharding is "
              "described in DESIGN.md but not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2607_21150_amd import inputs as I
    from paper_2607_21150_amd import pfmf

    t_gen = time.perf_counter()
    d = I.make_inputs(args.config, args.variant)
    mesh = d["mesh"]
    print(f"[bench] inputs {args.config}/{args.variant}: {mesh.n_dof} DoFs, {mesh.n_q} qps, "
          f"generated in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", torch.float64)
    ctx = pfmf.Context.from_inputs(d)
    z, dz, v = dev(d["z"]), dev(d["dz"]), dev(d["v_top"])
    r = torch.empty_like(z)
    y = torch.empty_like(z)
    gz = torch.empty_like(z)
    gp = torch.empty((len(d["phases"]), 3), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    ys = torch.empty_like(z)
    dz32 = dz.float()
    y32 = torch.empty_like(dz32)
    b32 = torch.empty_like(dz32)
    x32 = torch.empty_like(dz32)
    ctx.linearize(z)
    ctx.apply_jacobian_f32(0, dz32, b32)

    # Order within a step: the linearisation synchronises the host (power iteration), so the
    # queue is empty after it; the V-cycle follows it (its many launches dwarf the first
    # launch's host latency), and the single applies are enqueued while earlier work still
    # runs, so their event pairs measure device time, not host launch latency.
    ops = {
        "linearize": lambda: ctx.linearize(z),
        "vcycle": lambda: ctx.pmg_vcycle(b32, x32),
        "fp32_apply": lambda: ctx.apply_jacobian_f32(0, dz32, y32),
        "residual": lambda: ctx.apply_residual(z, r),
        "jacobian": lambda: ctx.apply_jacobian(z, dz, y),
        "adjoint": lambda: ctx.apply_adjoint(z, v, gz, gp),
        "jacobian_stored": lambda: ctx.apply_jacobian_lin(dz, ys),
    }
    for _ in range(args.warmup):
        for f in ops.values():
            f()
    torch.cuda.synchronize()
    ctx.check()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    ev = {k: [] for k in ops}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for k, f in ops.items():
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            f()
            b.record(stream)
            ev[k].append((a, b))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = {k: float(np.mean([a.elapsed_time(b) for a, b in ev[k]])) for k in ev}
    ms_min = {k: float(np.min([a.elapsed_time(b) for a, b in ev[k]])) for k in ev}
    ms_med = {k: float(np.median([a.elapsed_time(b) for a, b in ev[k]])) for k in ev}
    print(f"[bench] timed {args.steps} steps in {wall:.2f} s: {ms}", file=sys.stderr, flush=True)

    # errors against the oracle on every node of the mesh (FP64 bar 1e-12, FP32 1e-5)
    errs = {}
    try:
        if args.no_oracle:
            raise RuntimeError("skipped (--no-oracle)")
        from oracle import pyoracle
        pyoracle.build(force=False)
        orc = pyoracle.Oracle.from_inputs(d)
        t_or = time.perf_counter()
        errs["residual"] = whole_mesh_err(r.cpu().numpy(), orc.residual(d["z"]))
        jref = orc.jacobian(d["z"], d["dz"])
        errs["jacobian"] = whole_mesh_err(y.cpu().numpy(), jref)
        errs["fp32_apply"] = whole_mesh_err(y32.double().cpu().numpy(), jref)
        errs["jacobian_stored"] = whole_mesh_err(ys.cpu().numpy(), jref)
        del jref
        errs["adjoint"] = whole_mesh_err(gz.cpu().numpy(), orc.adjoint(d["z"], d["v_top"])[0])
        errs["nodes_compared"] = mesh.n_nodes
        print(f"[bench] whole-mesh oracle comparison in {time.perf_counter() - t_or:.1f} s: {errs}",
              file=sys.stderr, flush=True)
    except Exception as exc:  # the oracle is a checker; its absence does not stop the benchmark
        errs["error"] = str(exc)

    copy = copy_probe(torch)
    print(f"[bench] copy probe {copy}", file=sys.stderr, flush=True)

    # DoF/s and GB/s from the median apply time (the mean, min and median are all reported)
    t_jac = ms_med["jacobian"] * 1e-3
    value = mesh.n_dof / t_jac
    bj = alg_bytes(mesh, "jacobian")
    achieved = bj / t_jac / 1e9
    counters = measured_counters(args.config + "/" + args.variant)
    traffic = counters.get("hbm_bytes_per_apply")
    kname = {2: "pfmf::k_op64_q2r<1, false> + pfmf::k_gather_ext<double, 5>: one "
                "launch over all bricks, then the node gather",
             3: "pfmf::k_op64_q3<1, true, false, false, false, false> + pfmf::k_gather_ext<double, 7>: one "
                "launch over all bricks, then the node gather",
             4: "pfmf::k_op64_q4<1, false, false, false, true, false> + pfmf::k_gather_ext<double, 5>: one launch over "
                "all elements, then the node gather"}.get(mesh.p, f"pfmf::k_op64<1, {mesh.p + 1}, {mesh.p + 1}>")
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(d, args.cpu_seconds)
    out = {
        "metric": "Jacobian-apply DoFs/s (Q2/Q3 hex) FP64 vs FP32 p-MG, % HBM roofline, rel err",
        "value": value,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": float(sum(ms.values())),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.config} Q{mesh.p} hex {mesh.nx}x{mesh.ny}x{mesh.nz} elements, 1 mm cube, "
                        f"{mesh.n_dof} DoFs, {mesh.n_q} quadrature points, particle volume fraction "
                        f"{d['vol_frac']:.3f}, loading '{args.variant}' (e0={d['e0']})",
            "p": mesh.p, "elements": [mesh.nx, mesh.ny, mesh.nz], "n_dof": mesh.n_dof, "n_q": mesh.n_q,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": f"{kname} (one Jacobian apply; bytes and time per apply)",
            "alg_bytes_per_apply": bj,
            "copy_probe_gbs": copy["gbs"],
        },
        # achieved FP64 FLOP/s of the Jacobian apply: counted FLOPs per apply (rocprofv3, the
        # committed summary of these kernel sources) over the median apply time, against the FP64
        # peak; null when the summary does not match the sources
        "alu": ({"bound": "alu", "unit": "TFLOP/s",
                 "achieved": (counters["valu_fp64_flops_per_apply"] + counters["mfma_f64_flops_per_apply"])
                 / t_jac / 1e12,
                 "peak": FP64_VEC_PEAK_TFLOPS,
                 "frac": (counters["valu_fp64_flops_per_apply"] + counters["mfma_f64_flops_per_apply"])
                 / t_jac / 1e12 / FP64_VEC_PEAK_TFLOPS,
                 "valu_fp64_flops_per_apply": counters["valu_fp64_flops_per_apply"],
                 "mfma_f64_flops_per_apply": counters["mfma_f64_flops_per_apply"]}
                if "valu_fp64_flops_per_apply" in counters and "mfma_f64_flops_per_apply" in counters else None),
        "cpu_baseline": cpu,
        "ms": ms,
        "ms_min": ms_min,
        "ms_median": ms_med,
        "dofs_per_s": {k: mesh.n_dof / (ms_med[k] * 1e-3) for k in ("residual", "jacobian", "adjoint",
                                                                     "fp32_apply", "jacobian_stored")},
        "gbs_alg": {k: alg_bytes(mesh, k) / (ms_med[k] * 1e-3) / 1e9 for k in ("residual", "jacobian", "adjoint",
                                                                                  "fp32_apply", "jacobian_stored")},
        # the FP64 Jacobian from the linearisation stored by pf_linearize (same operator at the same
        # z, record read instead of the point state recomputed): HBM-bound, reported beside the
        # recompute apply above, which is `value`
        "roofline_jacobian_stored": {
            "bound": "hbm",
            "achieved": alg_bytes(mesh, "jacobian_stored") / (ms_med["jacobian_stored"] * 1e-3) / 1e9,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": alg_bytes(mesh, "jacobian_stored") / (ms_med["jacobian_stored"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "alg_bytes_per_apply": alg_bytes(mesh, "jacobian_stored"),
            "bytes_read_and_written": stored_bytes(mesh, "jacobian_stored"),
        },
        "roofline_fp32_apply": {
            "bound": "hbm",
            "achieved": alg_bytes(mesh, "fp32_apply") / (ms_med["fp32_apply"] * 1e-3) / 1e9,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": alg_bytes(mesh, "fp32_apply") / (ms_med["fp32_apply"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "alg_bytes_per_apply": alg_bytes(mesh, "fp32_apply"),
            "bytes_read_and_written": stored_bytes(mesh, "fp32_apply"),
        },
        "fp32_over_fp64_apply_speedup": ms_med["jacobian"] / ms_med["fp32_apply"],
        "fp32_over_stored_fp64_speedup": ms_med["jacobian_stored"] / ms_med["fp32_apply"],
        "rel_err_vs_oracle": errs,
        "paper_context": PAPER_CONTEXT,
    }
    newton = not args.no_newton
    if args.secondary or newton or args.branches or args.geometry or args.table:
        del ctx, z, dz, v, r, y, gz, dz32, y32, b32, x32, ys
        torch.cuda.empty_cache()
    if args.branches:
        out["branches"] = branches_leg(torch, I, pfmf, args.branches)
        print(f"[bench] branches {out['branches']}", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    if args.geometry:
        out["geometry"] = geometry_leg(torch, I, pfmf, args.geometry, with_box=args.geometry_box)
        print(f"[bench] geometry {out['geometry']}", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    if args.table:
        out["table"] = table_leg(torch, I, pfmf, args.table)
        print(f"[bench] table {out['table']}", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    if args.secondary:
        out["secondary"] = secondary_leg(torch, I, pfmf, args.secondary)
        print(f"[bench] secondary {out['secondary']}", file=sys.stderr, flush=True)
    if newton:
        torch.cuda.empty_cache()
        out["newton"] = newton_leg(torch, I, pfmf, args.newton_config, with_cg=True, h_levels=True)
    if newton and args.newton_all:
        if args.newton_branches_config:
            torch.cuda.empty_cache()
            # the third example's matrix needs a stronger smoother than the defaults
            out["newton_branches"] = newton_leg(torch, I, pfmf, args.newton_branches_config, "ex3", cheb_degree=12,
                                                coarse_sweeps=64, restart=60, h_levels=True)
        if args.newton_curved_config:
            torch.cuda.empty_cache()
            # the curved mesh, like the third example's matrix, needs a stronger smoother than the
            # defaults (which stall near 2e-7 of the initial residual at C5)
            out["newton_curved"] = newton_leg(torch, I, pfmf, args.newton_curved_config, geometry="curved",
                                              cheb_degree=6, coarse_sweeps=64, restart=60, h_levels=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
