"""Throughput of the THC-oo-K exchange build (K^k for all k plus E_x) on one GPU.

Default workload (the metric's configuration): the 24-cell batch, 2 x {8, 16,
24, 48 atoms} x {1^3, 2^3, 3^3} k-meshes, 4 Gaussian functions per atom
(N = 32 .. 192), n_occ = 0.44 N, N_ISDF = 2.2 N, grids at 4.5 points/bohr.
One step = the whole batch of K-builds through one exx_build_batched call
(a captured HIP graph or concurrent lanes, whichever is faster; autotuned
tiles) in the mixed precision mode (FP64 fit, FP32 storage of the fitted
functions and transforms, FP64 Cholesky, solve arithmetic, Coulomb
contraction on the FP64 matrix cores, FP64 K and E_x; no refinement step). It is compared
with 24 sequential plain-FP64 builds of the same cells, and every cell's E_x
and K are checked against the stored FP64 oracle values (tests/golden/
config4.json, written by the oracle alone) at |dE_x| <= 1e-5 Ha/cell and
max|dK| <= 1e-6. Inputs are seeded, synthetic and resident in HBM before the
timed region.

`value` = 24 / (seconds per batched step). `paths` also carries the batch in
F32 and F64 and the single-cell builds of the 48-atom four-ring cell on the
2x2x2 and 3x3x3 meshes (N = 192, n_occ = 84, grid 60x75x54, N_ISDF = 420) in
every precision, with the split-BF16 contraction in MIXED and F32, each
against its stored oracle K and E_x, and the shared-xi fit (timed; its E_x
against the per-transfer oracle's shows the fit's own error).

Options: --steps K --warmup W --gpus N (N must be 1) --no-cpu --record PATH (append
JSONL run records) --profile
(the profiler's target, no JSON: the mixed batch twice and a 1 GiB copy; with
--phases, the tuning batch, then the 24 single builds with serial phase events
that the roofline is computed from, and the copy; with
--workload rings-k2 | rings-k3, two builds per precision of that cell and the
copy; with --potentials and a ring workload, the exchange gradient and the
robust-fit K instead); --workload rings-k2 | rings-k3 | select-k4 print a single
leg; --workload nk-series times the ring cell's build on 1^3..4^3 k-meshes;
--workload ao-k times THC-AO-K (fit once, K per iteration) on the 2x2x2 ring cell.
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
GOLDEN = os.path.join(ROOT, "tests", "golden")

METRIC = "K-builds/sec (all k) vs plain FP64 GPU at |ΔE_x|≤1e-5 Ha/cell; MFMA %"
PEAK = {"hbm_GBs": 8000.0, "fp64_TF": 78.6, "fp32_TF": 157.3}  # MI355X published dense peaks
GATE_E, GATE_K = 1e-5, 1e-6


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# algorithmic work
# ---------------------------------------------------------------------------
def n_pairs(kmesh):
    """Transfers m with m <= -m on the mesh (one per conjugate pair)."""
    N = kmesh
    cnt = 0
    for m in range(N[0] * N[1] * N[2]):
        m1, m2, m3 = m // (N[1] * N[2]), (m // N[2]) % N[1], m % N[2]
        b = (((N[0] - m1) % N[0]) * N[1] + (N[1] - m2) % N[1]) * N[2] + (N[2] - m3) % N[2]
        cnt += m <= b
    return cnt


def real_path(cell):
    return all(n <= 2 for n in cell.kmesh)


def work(cell, prec):
    """Per-build work of each phase: {phase: (unit, executed, plain)}.

    `executed` counts what the kernels do after the method's exact identities:
    on meshes with every N_i <= 2 the unphased metric and right-hand side are
    real (real solve by the triangular inverse factor, N_ISDF (N_ISDF + 1)/2
    multiply-adds per grid point; half-grid transform; real Coulomb sum over
    n1 n2 (n3/2 + 1) points, lower triangle); elsewhere one transfer of each
    pair (m, -m) is fitted, transformed and contracted (complex, Gauss's
    three-product form on the FP64 matrix cores: 6 flops per complex
    multiply-add; triangular solve; lower triangle of V). `plain` counts the
    plain method: Gamma 8 N_k N_I n_o N_g, solve 8 N_k N_I^2 N_g, Coulomb
    (Hermitian) 4 N_k N_I^2 N_g, one read and one write of the N_k N_I N_g
    intermediate for the k-correlation and the transform.
    """
    nk, ng, no, na, ni = cell.N_k, cell.N_g, cell.n_occ, cell.n_ao, cell.n_isdf
    cs = 16 if prec in ("f64", "mixed") else 8   # Gamma / Z element (complex)
    cx = 16 if prec == "f64" else 8              # xi / transform element (complex)
    sv = {
        "gamma": ("flop", 8.0 * nk * ni * no * ng),
        "kcorr": ("byte", 2.0 * nk * ni * ng * cs),
        "solve": ("flop", 8.0 * nk * ni * ni * ng),
        "fft": ("byte", 2.0 * nk * ni * ng * cx),
        "coulomb": ("flop", 4.0 * nk * ni * ni * ng),
        "K": ("flop", 8.0 * nk * (na * ni * ni + na * na * ni)),
    }
    cg = 8.0 if prec == "f32" else 6.0
    ex = {"gamma": cg * nk * ni * no * ng, "K": 8.0 * nk * (na * ni * ni + na * na * ni)}
    if real_path(cell):
        n1, n2, n3 = cell.grid
        ngh = n1 * n2 * (n3 // 2 + 1)
        gam = 8 if prec == "f32" else 16
        zr = 4 if prec == "f32" else 8
        xr = 8 if prec == "f64" else 4
        xc = 16 if prec == "f64" else 8
        ex.update({
            "kcorr": nk * ni * ng * (gam + zr),
            "solve": 1.0 * ni * (ni + 1) * nk * ng,
            "fft": nk * ni * (ng * xr + ngh * xc),
            "coulomb": 2.0 * nk * ni * ni * ngh,
        })
        if prec == "f32":
            ex["gamma"] = 8.0 * nk * ni * no * ng  # Gamma and Z~ in one FP32-core kernel
    else:
        npr = n_pairs(cell.kmesh)
        ex.update({
            "kcorr": (nk + npr) * ni * ng * cs,
            "solve": 3.0 * npr * ni * (ni + 1) * ng,
            "fft": 2.0 * npr * ni * ng * cx,
            "coulomb": 3.0 * npr * ni * (ni + 1) * ng,
        })
    return {p: (sv[p][0], ex[p], sv[p][1]) for p in sv}


FP64_CORES = {"f64": {"gamma", "solve", "coulomb", "K"}, "mixed": {"gamma", "solve", "coulomb", "K"},
              "f32": {"solve", "coulomb", "K"}}

KERNELS = {  # dominant kernel(s) of each phase, real path / paired path
    "gamma": ("zgemm_nn_mfma (FP64) or gamma_kcorr_kernel (F32)", "zgemm_nn_mfma / cgemm FP32 cores"),
    "solve": ("dgemm_nn_mfma (triangular W)", "zgemm_nn_mfma (triangular W)"),
    "coulomb": ("coulomb_kernel_t64", "coulomb_kernel_f64 / coulomb_kernel_f32"),
    "fft": ("fft_yz_half2_kernel + fft_x", "fft_yz + fft_x"),
    "kcorr": ("kcorr_real_kernel", "kcorr_kernel"),
}


# HBM bytes the dominant phase's kernels moved in one 24-cell MIXED batch, from
# the rocprofv3 FETCH_SIZE and WRITE_SIZE runs of `bench.py --profile` (scaled by
# the counters' reading for a plain 1 GiB copy; profiles/hbm_traffic_batch24_mixed.md).
# Valid only while the kernels' source file is unchanged (SHA-256 below).
TRAFFIC = {
    "solve": {"source": "paper_2304_05505_amd/csrc/gemm_mfma.hip",
              "sha256": "20b9f74537d768698d899cf87c6d402ee90c1e5f49d29311f9b3873cd09a23ef",
              "bytes": 344.59e9, "launches": 38,
              "kernels": ["zgemm_nn_mfma<double, float, 2, 2, 0, 0, 1>",
                          "dgemm_nn_mfma<double, float, 1, 0>"]},
}


def traffic_for(phase):
    import hashlib

    t = TRAFFIC.get(phase)
    if not t:
        return None
    with open(os.path.join(ROOT, t["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != t["sha256"]:
            return None
    return {"bytes_per_batch": t["bytes"], "launches": t["launches"],
            "bytes_per_launch": t["bytes"] / t["launches"], "kernels": t["kernels"],
            "counted": "FETCH_SIZE x2.0 + WRITE_SIZE x1.0 (1 GiB copy calibration); includes "
                       "lines served by the last-level cache"}


def phase_rate(p, phase_ms, work_exec, work_plain, units, prec):
    """Achieved rate of phase p (executed and plain-method work counts) over its summed time."""
    s = phase_ms[p] / 1e3
    if units[p] == "byte":
        a, a_sv = work_exec[p] / s / 1e9, work_plain[p] / s / 1e9
        out = {"bound": "hbm", "achieved": a, "peak": PEAK["hbm_GBs"], "unit": "GB/s",
               "frac": a / PEAK["hbm_GBs"]}
    else:
        a, a_sv = work_exec[p] / s / 1e12, work_plain[p] / s / 1e12
        peak = PEAK["fp64_TF"] if p in FP64_CORES[prec] else PEAK["fp32_TF"]
        out = {"bound": "mfma", "achieved": a, "peak": peak, "unit": "TFLOP/s", "frac": a / peak}
    out.update({"phase_ms": phase_ms[p], "work_executed": work_exec[p],
                "work_plain": work_plain[p], "achieved_plain_count": a_sv,
                "frac_plain_count": a_sv / out["peak"]})
    return out


def roofline(phase_ms, work_exec, work_plain, units, prec):
    """Roofline of the phase with the largest summed time. phase_ms: {phase: ms};
    work_*: {phase: amount} summed over the same builds."""
    best = max((p for p in phase_ms if p in work_exec and phase_ms[p] > 0), key=lambda p: phase_ms[p])
    out = phase_rate(best, phase_ms, work_exec, work_plain, units, prec)
    out.update({"traffic": traffic_for(best), "phase": best})
    return out


# ---------------------------------------------------------------------------
# stored oracle values
# ---------------------------------------------------------------------------
def load_json(name):
    p = os.path.join(GOLDEN, name)
    return json.load(open(p)) if os.path.exists(p) else None


def load_npz(name):
    p = os.path.join(GOLDEN, name)
    if not os.path.exists(p):
        return None
    with np.load(p, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def cpu_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model or platform.processor()


# ---------------------------------------------------------------------------
# inputs
# ---------------------------------------------------------------------------
def cell_inputs(h, exx, torch, cell, dev, pts=None):
    """Orbitals on the grid (generated on the GPU), points (given, else GPU QRCP),
    orbital and basis values at the points; all resident on the device."""
    import synth
    from synth.fast import orbitals_on_grid_torch

    psi = orbitals_on_grid_torch(cell, synth.orbital_coeffs(cell), dev)
    c = exx.make_cell(cell.L, cell.grid, cell.kmesh, cell.n_occ, cell.n_ao, cell.n_isdf)
    if pts is None:
        pts_t = torch.empty((cell.n_isdf,), dtype=torch.int32, device=dev)
        npiv = torch.empty((1,), dtype=torch.int32, device=dev)
        exx.exx_select_points(h, c, psi, pts_t, npiv)
        pts = pts_t.cpu().numpy().astype(np.int64)
    else:
        pts = np.asarray(pts, dtype=np.int64)
        pts_t = torch.from_numpy(pts.astype(np.int32)).to(dev)
    ao = np.stack([synth.ao_at_points(cell, n, pts) for n in range(cell.N_k)])
    return {
        "cell": c,
        "psi64": psi,
        "occ_pts": psi[:, :, pts_t.long()].permute(0, 2, 1).contiguous(),
        "ao_pts": torch.from_numpy(np.ascontiguousarray(np.transpose(ao, (0, 2, 1)))).to(dev),
        "pts": pts_t,
        "pts_np": pts,
    }


def outputs(torch, cell, dev):
    return {"K": torch.empty((cell.N_k, cell.n_ao, cell.n_ao), dtype=torch.complex128, device=dev),
            "Ex": torch.empty((1,), dtype=torch.float64, device=dev),
            "rank": torch.empty((cell.N_k,), dtype=torch.int32, device=dev)}


def psi_for(t, prec, torch):
    if prec in ("f32", "bf16"):
        if "psi32" not in t:
            t["psi32"] = t["psi64"].to(torch.complex64)
        return t["psi32"]
    return t["psi64"]


def time_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


# ---------------------------------------------------------------------------
# single-cell legs (the 48-atom ring cell on 2x2x2 and 3x3x3)
# ---------------------------------------------------------------------------
# (label, precision, contraction form, fit) of the single-cell legs
VARIANTS = (("f64", "f64", 0, 0), ("mixed", "mixed", 0, 0), ("f32", "f32", 0, 0),
            ("bf16", "bf16", 0, 0), ("mixed+bf16x3", "mixed", 3, 0), ("f32+bf16x3", "f32", 3, 0),
            ("f64-shared", "f64", 0, 1), ("mixed-shared", "mixed", 0, 1))
CONTRACTION_NAMES = {0: "auto (FP64 matrix cores; BF16 in bf16)", 1: "FP64 matrix cores",
                     2: "BF16 matrix cores", 3: "split BF16 (three products)"}


def ring_leg(config, args, h, exx, torch, dev):
    import synth

    cell = synth.make_config(config)
    tag = f"rings-k{cell.kmesh[0]}"
    gold = load_json(f"config{config}.json")
    goldK = load_npz(f"config{config}_K.npz")
    t0 = time.perf_counter()
    t = cell_inputs(h, exx, torch, cell, dev, pts=gold["pts"] if gold else None)
    torch.cuda.synchronize()
    log(f"[{tag}] inputs in {time.perf_counter() - t0:.1f} s")
    res = {}
    for label, prec, form, fit in VARIANTS:
        o = outputs(torch, cell, dev)
        h.set_contraction(form)
        h.set_fit(fit)

        def step():
            exx.exx_build(h, t["cell"], exx.PREC[prec], psi_for(t, prec, torch), t["occ_pts"],
                          t["ao_pts"], t["pts"], o["K"], o["Ex"], o["rank"])

        s = time_steps(step, max(1, args.steps), max(1, args.warmup), torch)
        h.set_timing(True, serial=True)
        step()
        torch.cuda.synchronize()
        ph = {k: v[0] for k, v in h.phase_times().items()}
        h.set_timing(False)
        h.set_contraction(exx.EXX_CONTRACT_AUTO)
        h.set_fit(exx.EXX_FIT_PER_Q)
        r = {"ms_per_build": s * 1e3, "builds_per_s": 1.0 / s, "Ex": float(o["Ex"].cpu()[0]),
             "precision": prec, "contraction": CONTRACTION_NAMES[form],
             "fit": "shared" if fit else "per transfer", "phases_ms": ph}
        if gold is not None and goldK is not None and "K" in goldK:
            K = o["K"].cpu().numpy()
            if fit:
                # the shared fit is another approximation: its distance from the
                # per-transfer oracle is the fit's own error, not a parity figure
                r["Ex_minus_per_transfer_oracle"] = r["Ex"] - gold["Ex"]
            else:
                r["dEx_vs_oracle"] = abs(r["Ex"] - gold["Ex"])
                r["maxdK_vs_oracle"] = float(np.abs(K - goldK["K"]).max())
                r["meets_gate"] = bool(r["dEx_vs_oracle"] <= GATE_E
                                       and r["maxdK_vs_oracle"] <= GATE_K)
        res[label] = r
        log(f"[{tag}] {label}: {s * 1e3:.2f} ms/build, E_x {r['Ex']:.10f}" +
            (f", |dEx| {r['dEx_vs_oracle']:.2e}, max|dK| {r['maxdK_vs_oracle']:.2e}"
             if "dEx_vs_oracle" in r else ""))
    for label in res:
        res[label]["speedup_vs_f64"] = res["f64"]["ms_per_build"] / res[label]["ms_per_build"]
    # the gradient and robust calls: on the 2x2x2 cell always; on the 3x3x3 cell
    # (three N_k N_I N_g c128 arrays, 132 GB, beside the build's scratch) only
    # when that workload is asked for by itself
    if config == 2 or args.workload == "rings-k3":
        res.update(potential_legs(args, h, exx, torch, dev, cell, t, res["f64"]["ms_per_build"],
                                  tag))
    return {"workload": f"48-atom four-ring cell, {'x'.join(map(str, cell.kmesh))} k-mesh, N=192, "
                        f"n_occ=84, grid 60x75x54, N_ISDF=420", "paths": res}


def potential_legs(args, h, exx, torch, dev, cell, t, f64_ms, tag):
    """The FP64 calls that add the potentials of the fitted functions to a build:
    the exchange gradient (K, E_x and Kgrad) and the robust-fit K, each timed as
    one whole call (its build included) and against the fused FP64 build and the
    stage-wise one (fit, Coulomb, K: the route these calls take, since they need
    xi^m of every transfer)."""
    from synth.fast import ao_on_grid_torch

    ao_grid = torch.stack([ao_on_grid_torch(cell, n, dev) for n in range(cell.N_k)]).contiguous()
    out = {}
    o = outputs(torch, cell, dev)
    Kg = torch.empty_like(o["K"])
    nk, ni, ng = cell.N_k, cell.n_isdf, int(np.prod(cell.grid))
    xi = torch.empty((nk, ni, ng), dtype=torch.complex128, device=dev)
    S = torch.empty((nk, ni, ni), dtype=torch.complex128, device=dev)
    V = torch.empty_like(S)

    def stagewise():
        # the build route of these calls: xi^m of every transfer formed
        exx.exx_isdf_fit(h, t["cell"], exx.EXX_F64, t["psi64"], t["occ_pts"], t["pts"], xi, S,
                         o["rank"])
        exx.exx_coulomb_V(h, t["cell"], exx.EXX_F64, xi, t["pts"], V)
        exx.exx_build_K(h, t["cell"], exx.EXX_F64, t["ao_pts"], t["occ_pts"], V, o["K"], o["Ex"])

    s = time_steps(stagewise, max(1, min(args.steps, 3)), 1, torch)
    out["f64-stagewise"] = {"ms_per_build": s * 1e3, "ratio_to_f64_build": s * 1e3 / f64_ms,
                            "precision": "f64", "Ex": float(o["Ex"].cpu()[0])}
    log(f"[{tag}] f64-stagewise: {s * 1e3:.2f} ms/build ({s * 1e3 / f64_ms:.2f}x the fused build)")
    del xi, S, V
    stage_ms = s * 1e3
    calls = {
        "f64-gradient": lambda: exx.exx_exchange_gradient(
            h, t["cell"], t["psi64"], t["occ_pts"], t["ao_pts"], ao_grid, t["pts"], o["K"], Kg,
            o["Ex"], o["rank"]),
        "f64-robust": lambda: exx.exx_build_robust(
            h, t["cell"], t["psi64"], t["occ_pts"], t["ao_pts"], ao_grid, t["pts"], o["K"],
            o["Ex"], o["rank"]),
        "mixed-gradient": lambda: exx.exx_exchange_gradient(
            h, t["cell"], t["psi64"], t["occ_pts"], t["ao_pts"], ao_grid, t["pts"], o["K"], Kg,
            o["Ex"], o["rank"], prec=exx.EXX_MIXED),
        "mixed-robust": lambda: exx.exx_build_robust(
            h, t["cell"], t["psi64"], t["occ_pts"], t["ao_pts"], ao_grid, t["pts"], o["K"],
            o["Ex"], o["rank"], prec=exx.EXX_MIXED),
    }
    for label, fn in calls.items():
        s = time_steps(fn, max(1, min(args.steps, 3)), 1, torch)
        out[label] = {"ms_per_call": s * 1e3, "ratio_to_f64_build": s * 1e3 / f64_ms,
                      "ratio_to_f64_stagewise_build": s * 1e3 / stage_ms,
                      "Ex": float(o["Ex"].cpu()[0]), "precision": label.split("-")[0]}
        log(f"[{tag}] {label}: {s * 1e3:.2f} ms/call ({s * 1e3 / f64_ms:.2f}x the fused FP64 "
            f"build, {s * 1e3 / stage_ms:.2f}x the stage-wise one)")
    del ao_grid, Kg
    torch.cuda.empty_cache()
    if not args.no_cpu:
        out["f64-gradient"]["cpu_oracle"] = gradient_cpu_sample(h, exx, torch, dev, tag)
    return out


def gradient_cpu_sample(h, exx, torch, dev, tag):
    """The gradient oracle timed beside the GPU call on one small cell of the
    batch (the 8-atom 2x2x2 cell: N 32, n_occ 14, N_ISDF 70, 36x45x32 grid):
    one oracle call (thc_oo_k_gradient: fit, potentials, correlations, AO
    products, all FP64 on the host) against the median GPU call."""
    import synth
    from oracle import select, thc
    from oracle._threads import WORKERS

    cell = [c for c in synth.make_batch_cells() if c.name == "batch1-a8-k2"][0]
    psi = synth.orbitals_on_grid(cell, synth.orbital_coeffs(cell))
    phi = np.stack([synth.ao_on_grid(cell, n) for n in range(cell.N_k)])
    pts, _ = select.select_points(psi, cell.n_isdf)
    t0 = time.perf_counter()
    ref = thc.thc_oo_k_gradient(cell.L, cell.grid, cell.kmesh, psi, phi, pts)
    t_cpu = time.perf_counter() - t0
    nk, na, ni = cell.N_k, cell.n_ao, len(pts)
    ao = np.stack([phi[n][:, pts] for n in range(nk)])
    c = exx.make_cell(cell.L, cell.grid, cell.kmesh, cell.n_occ, na, ni)
    args_t = (torch.from_numpy(psi).to(dev),
              torch.from_numpy(np.ascontiguousarray(np.transpose(psi[:, :, pts], (0, 2, 1)))).to(dev),
              torch.from_numpy(np.ascontiguousarray(np.transpose(ao, (0, 2, 1)))).to(dev),
              torch.from_numpy(np.ascontiguousarray(phi)).to(dev),
              torch.from_numpy(np.asarray(pts, dtype=np.int32)).to(dev))
    K = torch.empty((nk, na, na), dtype=torch.complex128, device=dev)
    Kg = torch.empty_like(K)
    Ex = torch.empty((1,), dtype=torch.float64, device=dev)
    rank = torch.empty((nk,), dtype=torch.int32, device=dev)
    s = time_steps(lambda: exx.exx_exchange_gradient(h, c, *args_t, K, Kg, Ex, rank), 5, 1, torch)
    dG = float(np.abs(Kg.cpu().numpy() - ref["Kgrad"]).max() / np.abs(ref["Kgrad"]).max())
    log(f"[{tag}] gradient on {cell.name}: oracle {t_cpu:.1f} s on the host, GPU {s * 1e3:.2f} ms, "
        f"rel max|dKgrad| {dG:.1e}")
    return {"cell": cell.name, "oracle_s": t_cpu, "gpu_ms": s * 1e3, "cores": WORKERS,
            "cpu_model": cpu_info(), "rel_max_dKgrad": dG}


# ---------------------------------------------------------------------------
# the 24-cell batch
# ---------------------------------------------------------------------------
def batch_errors(items, gold, goldK):
    """Per-cell |dE_x| and max|dK| (stored oracle entries and diagonals)."""
    dE, dK = [], []
    for i, it in enumerate(items):
        g = gold["cells"][i]
        K = it["K"].cpu().numpy()
        idx = goldK[f"idx_{i}"]
        d1 = np.abs(K[idx[:, 0], idx[:, 1], idx[:, 2]] - goldK[f"val_{i}"]).max()
        diag = np.stack([np.diagonal(K[n]) for n in range(K.shape[0])])
        d2 = np.abs(diag - goldK[f"diag_{i}"]).max()
        dE.append(abs(float(it["Ex"].cpu()[0]) - g["Ex"]))
        dK.append(float(max(d1, d2)))
    return dE, dK


def batch_leg(args, h, exx, torch, dev):
    import synth

    cells = synth.make_batch_cells()
    gold = load_json("config4.json")
    goldK = load_npz("config4_K.npz")
    if gold is not None and [g["name"] for g in gold["cells"]] != [c.name for c in cells]:
        gold = goldK = None
    t0 = time.perf_counter()
    base = [cell_inputs(h, exx, torch, c, dev, pts=gold["cells"][i]["pts"] if gold else None)
            for i, c in enumerate(cells)]
    torch.cuda.synchronize()
    log(f"[batch24] inputs for 24 cells in {time.perf_counter() - t0:.1f} s "
        f"({'oracle' if gold else 'GPU QRCP'} points)")

    def items(prec):
        out = []
        for c, t in zip(cells, base):
            out.append(dict(cell=t["cell"], psi_grid=psi_for(t, prec, torch), occ_pts=t["occ_pts"],
                            ao_pts=t["ao_pts"], pts=t["pts"], **outputs(torch, c, dev)))
        return out

    seq = items("f64")

    def sequential_f64():
        for it in seq:
            exx.exx_build(h, it["cell"], exx.EXX_F64, it["psi_grid"], it["occ_pts"], it["ao_pts"],
                          it["pts"], it["K"], it["Ex"], it["rank"])

    stream = torch.cuda.Stream()
    modes = {"graph": exx.EXX_BATCH_GRAPH | exx.EXX_BATCH_TUNE,
             "lanes": exx.EXX_BATCH_CONCURRENT | exx.EXX_BATCH_TUNE}

    def batched(prec, its, mode):
        flags = modes[mode]

        def fn():
            stream.wait_stream(torch.cuda.current_stream())
            exx.exx_build_batched(h, its, exx.PREC[prec], flags, stream=stream)
            torch.cuda.current_stream().wait_stream(stream)
        return fn

    steps, warmup = max(1, args.steps), max(1, args.warmup)
    res = {}
    s_seq = time_steps(sequential_f64, steps, warmup, torch)
    log(f"[batch24] 24 sequential plain-FP64 builds: {s_seq * 1e3:.1f} ms")
    seq_mixed = items("mixed")

    def sequential_mixed():
        for it in seq_mixed:
            exx.exx_build(h, it["cell"], exx.EXX_MIXED, it["psi_grid"], it["occ_pts"],
                          it["ao_pts"], it["pts"], it["K"], it["Ex"], it["rank"])

    s_seq_mixed = time_steps(sequential_mixed, steps, warmup, torch)
    del seq_mixed
    log(f"[batch24] 24 sequential MIXED builds: {s_seq_mixed * 1e3:.1f} ms")
    seq_err = batch_errors(seq, gold, goldK) if gold else None
    its_by_prec = {}
    for prec in ("mixed", "f32", "f64"):
        its = items(prec)
        its_by_prec[prec] = its
        t_mode = {}
        for mode in modes:
            t_mode[mode] = time_steps(batched(prec, its, mode),
                                      steps if prec == "mixed" else max(1, steps // 2), warmup, torch)
            log(f"[batch24] batched {prec} ({mode}): {t_mode[mode] * 1e3:.1f} ms")
        mode = min(t_mode, key=t_mode.get)
        batched(prec, its, mode)()  # the outputs checked below come from the reported mode
        torch.cuda.synchronize()
        s = t_mode[mode]
        r = {"seconds": s, "builds_per_s": 24.0 / s, "speedup_vs_sequential_f64": s_seq / s,
             "mode": mode, "seconds_by_mode": t_mode}
        if prec == "mixed":
            r["speedup_vs_sequential_same_precision"] = s_seq_mixed / s
        if gold:
            dE, dK = batch_errors(its, gold, goldK)
            r.update({"max_dEx_vs_oracle": max(dE), "max_dK_vs_oracle": max(dK),
                      "cells_meeting_gate": int(sum(e <= GATE_E and k <= GATE_K
                                                    for e, k in zip(dE, dK))),
                      "dEx_per_cell": dE, "dK_per_cell": dK})
        res[prec] = r
        log(f"[batch24] batched {prec}: {s * 1e3:.1f} ms ({s_seq / s:.2f}x sequential FP64)" +
            (f", max|dEx| {r['max_dEx_vs_oracle']:.2e}, max|dK| {r['max_dK_vs_oracle']:.2e}, "
             f"{r['cells_meeting_gate']}/24 cells in the gate" if gold else ""))
    seq_r = {"seconds": s_seq, "builds_per_s": 24.0 / s_seq,
             "sequential_mixed_seconds": s_seq_mixed}
    if seq_err:
        seq_r.update({"max_dEx_vs_oracle": max(seq_err[0]), "max_dK_vs_oracle": max(seq_err[1])})

    # per-phase event times of every cell's build (one untimed pass, same kernels
    # and shapes as the batch, the normally overlapping phases run one after
    # another so that each interval covers its own kernels) and the work counts
    phase_ms, wex, wsv, units = {}, {}, {}, {}
    its = its_by_prec["mixed"]
    h.set_timing(True, serial=True)
    for c, it in zip(cells, its):
        exx.exx_build(h, it["cell"], exx.EXX_MIXED, it["psi_grid"], it["occ_pts"], it["ao_pts"],
                      it["pts"], it["K"], it["Ex"], it["rank"])
        torch.cuda.synchronize()
        for p, (ms, _) in h.phase_times().items():
            phase_ms[p] = phase_ms.get(p, 0.0) + ms
        for p, (u, a, b) in work(c, "mixed").items():
            wex[p] = wex.get(p, 0.0) + a
            wsv[p] = wsv.get(p, 0.0) + b
            units[p] = u
    h.set_timing(False)
    return cells, res, seq_r, phase_ms, wex, wsv, units


# ---------------------------------------------------------------------------
# CPU oracle baseline
# ---------------------------------------------------------------------------
CPU_SAMPLE = ("batch0-a8-k1", "batch1-a8-k2", "batch3-a16-k1")


def cpu_baseline(cells):
    """Complete FP64 oracle K-builds (same steps as the GPU build) of three small
    cells of the batch, median of five passes (about 12 s of CPU work); scaled
    to the batch by the plain method's work (Gamma + solve + Coulomb flops of the
    plain-method count). Beside it, exact exchange (the direct oracle) on the
    first sample cell, timed once, with the fitted E_x of the same cell."""
    import synth
    from oracle import direct, select, thc
    from oracle._threads import WORKERS

    sample = [c for c in cells if c.name in CPU_SAMPLE]
    prepared = []
    for c in sample:
        psi = synth.orbitals_on_grid(c, synth.orbital_coeffs(c))
        pts, _ = select.select_points(psi, c.n_isdf)
        ao = np.stack([synth.ao_at_points(c, n, pts) for n in range(c.N_k)])
        prepared.append((c, psi, pts, ao))
    passes = []
    for _ in range(5):
        t0 = time.perf_counter()
        for j, (c, psi, pts, ao) in enumerate(prepared):
            o = thc.thc_oo_k(c.L, c.grid, c.kmesh, psi, pts, ao)
            if j == 0:
                e_thc = float(o["Ex"])
        passes.append(time.perf_counter() - t0)
    med = float(np.median(passes))
    # exact exchange (one FFT-Poisson solve per occupied pair density) on the
    # first sample cell: its cost, and what the fit at this N_ISDF misses there
    c0, psi0 = prepared[0][0], prepared[0][1]
    t0 = time.perf_counter()
    e_direct = float(direct.exchange_energy(c0.L, c0.grid, c0.kmesh, psi0))
    t_direct = time.perf_counter() - t0

    def w(c):
        sv = work(c, "f64")
        return sv["gamma"][2] + sv["solve"][2] + sv["coulomb"][2]

    scale = sum(w(c) for c in cells) / sum(w(c) for c, *_ in prepared)
    return {
        "value": 24.0 / (med * scale),
        "unit": "K-builds/s",
        "cores": WORKERS,
        "kind": "oracle",
        "cpu_model": cpu_info(),
        "sample": (f"complete oracle K-builds of {', '.join(c.name for c, *_ in prepared)} "
                   f"(median of 5 passes: {med:.2f} s for the {len(prepared)} cells, "
                   f"{len(prepared) / med:.3f} builds/s); scaled to the 24-cell batch by the "
                   f"plain method's flops (x{scale:.0f})"),
        "sample_seconds": passes,
        "direct_exchange": {"cell": c0.name, "seconds": t_direct, "Ex_direct": e_direct,
                            "Ex_thc": e_thc, "n_isdf": c0.n_isdf},
    }


# ---------------------------------------------------------------------------
# learned selection leg (unchanged workload)
# ---------------------------------------------------------------------------
def bench_select5(args):
    """Learned vs QRCP point selection at the 4x4x4 ring workload (2s + 2p basis,
    N 384, n_occ 84, grid 72x90x64, N_ISDF 420), each followed by the FP32 K-build
    at the chosen points: end-to-end time and the E_x difference."""
    import torch

    import synth
    from paper_2304_05505_amd import exx, mlp
    from synth.fast import orbitals_on_grid_torch

    dev = torch.device("cuda", 0)
    cell = synth.make_config(5)
    t0 = time.perf_counter()
    psi64 = orbitals_on_grid_torch(cell, synth.orbital_coeffs(cell), dev)
    psi32 = psi64.to(torch.complex64)
    torch.cuda.synchronize()
    log(f"[select5] orbitals generated in {time.perf_counter() - t0:.1f} s")
    nk, no, ng, ni, na = cell.N_k, cell.n_occ, cell.N_g, cell.n_isdf, cell.n_ao
    h = exx.Handle(0)
    c = exx.make_cell(cell.L, cell.grid, cell.kmesh, no, na, ni)
    w = mlp.load_weights()
    theta = torch.from_numpy(w["theta"]).to(dev)

    def timed(fn, reps):
        out, ts = None, []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return out, float(np.median(ts))

    def qrcp():
        pts = torch.empty((ni,), dtype=torch.int32, device=dev)
        npiv = torch.empty((1,), dtype=torch.int32, device=dev)
        exx.exx_select_points(h, c, psi64, pts, npiv)
        return pts

    # the fallback threshold for the 1e-5 Ha/cell fitted-exchange target, from
    # the calibration of the probe residual against the fitted-exchange error
    tau = mlp.tau_for(w, no)

    def learned(tau=tau):
        pts = torch.empty((ni,), dtype=torch.int32, device=dev)
        used, resid = exx.exx_select_points_mlp(h, c, psi64, w["norm"], theta, tau,
                                                int(w["n_probe"]), pts)
        return pts, used, resid

    learned()
    (pm, used, resid), t_mlp = timed(learned, 3)
    log(f"[select5] learned selection at the 1e-5 Ha/cell target (tau {tau:.2e}): "
        f"{t_mlp * 1e3:.1f} ms (fallback {used}, residual {resid:.4f})")
    # the network's own points (no fallback), for the comparison below
    (pn, _, resid_n), t_net = timed(lambda: learned(float("inf")), 3)
    pq, t_qrcp = timed(qrcp, 1)
    log(f"[select5] QRCP selection {t_qrcp * 1e3:.1f} ms")
    r = torch.empty((1,), dtype=torch.float64, device=dev)
    exx.exx_mlp_probe(h, c, psi64, pq, int(w["n_probe"]), int(w["probe_seed"]), r)
    resid_q = float(r.cpu()[0])

    def build(pts_t):
        pts = pts_t.cpu().numpy().astype(np.int64)
        ao = np.stack([synth.ao_at_points(cell, n, pts) for n in range(nk)])
        t_ao = torch.from_numpy(np.ascontiguousarray(np.transpose(ao, (0, 2, 1)))).to(dev)
        occ = psi64[:, :, pts_t.long()].permute(0, 2, 1).contiguous()
        K = torch.empty((nk, na, na), dtype=torch.complex128, device=dev)
        Ex = torch.empty((1,), dtype=torch.float64, device=dev)
        rank = torch.empty((nk,), dtype=torch.int32, device=dev)

        def run():
            exx.exx_build(h, c, exx.EXX_F32, psi32, occ, t_ao, pts_t, K, Ex, rank)

        run()
        _, t = timed(run, 2)
        return float(Ex.cpu()[0]), t

    ex_m, tb_m = build(pm)
    log(f"[select5] K-build (f32) at the selected points {tb_m * 1e3:.1f} ms, E_x {ex_m:.8f}")
    ex_n, tb_n = build(pn)
    log(f"[select5] K-build (f32) at the network's points {tb_n * 1e3:.1f} ms, E_x {ex_n:.8f}")
    ex_q, tb_q = build(pq)
    log(f"[select5] K-build (f32) at QRCP points {tb_q * 1e3:.1f} ms, E_x {ex_q:.8f}")
    pred_n = mlp.predicted_dex(w, no, resid_n)
    pred_q = mlp.predicted_dex(w, no, resid_q)
    out = {
        "metric": "end-to-end s: point selection + one K-build (all k), learned vs QRCP",
        "value": t_mlp + tb_m,
        "unit": "s",
        "n_gpus": 1,
        "higher_is_better": False,
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "48-atom four-ring cell, 4x4x4 k-mesh, 2s+2p (N=384), n_occ=84, "
                               "grid 72x90x64, N_ISDF=420", "N_k": nk, "N_g": ng},
        "target_dEx_Ha_per_cell": mlp.TARGET_DEX,
        "tau": tau,
        "learned": {"select_s": t_mlp, "build_s": tb_m, "Ex": ex_m, "probe_residual": resid,
                    "fallback": used},
        "network_points": {"select_s": t_net, "build_s": tb_n, "Ex": ex_n,
                           "probe_residual": resid_n, "predicted_dEx": pred_n,
                           "meets_target": bool(pred_n <= mlp.TARGET_DEX)},
        "qrcp": {"select_s": t_qrcp, "build_s": tb_q, "Ex": ex_q, "probe_residual": resid_q,
                 "predicted_dEx": pred_q, "meets_target": bool(pred_q <= mlp.TARGET_DEX)},
        "end_to_end_speedup": (t_qrcp + tb_q) / (t_mlp + tb_m),
        "end_to_end_speedup_network_points": (t_qrcp + tb_q) / (t_net + tb_n),
        "dEx_network_vs_qrcp": ex_n - ex_q,
    }
    print(json.dumps(out), flush=True)


def bench_nk_series(args):
    """The fused build of the 48-atom ring cell (configs 2 and 3: 60x75x54 grid,
    N 192, n_occ 84, N_ISDF 420) on 1^3, 2^3, 3^3 and 4^3 k-meshes, FP64 and
    MIXED, points by the GPU QRCP: time per build against N_k (the paper's
    K-build time grows linearly with the number of k-points)."""
    import torch

    import synth
    from paper_2304_05505_amd import exx

    dev = torch.device("cuda", 0)
    h = exx.Handle(0)
    rows = []
    for k in (1, 2, 3, 4):
        cell = synth.make_ring_series_cell(k)
        t = cell_inputs(h, exx, torch, cell, dev)
        o = outputs(torch, cell, dev)
        row = {"kmesh": [k, k, k], "N_k": cell.N_k}
        for prec in ("f64", "mixed"):
            def step():
                exx.exx_build(h, t["cell"], exx.PREC[prec], psi_for(t, prec, torch), t["occ_pts"],
                              t["ao_pts"], t["pts"], o["K"], o["Ex"], o["rank"])

            s = time_steps(step, max(1, min(args.steps, 3)), 1, torch)
            row[f"{prec}_ms"] = s * 1e3
            row[f"{prec}_ms_per_k"] = s * 1e3 / cell.N_k
            row[f"{prec}_Ex"] = float(o["Ex"].cpu()[0])
            log(f"[nk-series] {k}x{k}x{k}: {prec} {s * 1e3:.2f} ms/build "
                f"({s * 1e3 / cell.N_k:.2f} ms per k-point)")
        # one MIXED build with phase events, the overlapping phases serialised
        h.set_timing(True, serial=True)
        exx.exx_build(h, t["cell"], exx.EXX_MIXED, psi_for(t, "mixed", torch), t["occ_pts"],
                      t["ao_pts"], t["pts"], o["K"], o["Ex"], o["rank"])
        torch.cuda.synchronize()
        row["mixed_phases_ms"] = {p: ms for p, (ms, _) in h.phase_times().items()}
        h.set_timing(False)
        log(f"[nk-series] {k}x{k}x{k}: mixed phases " +
            ", ".join(f"{p} {ms:.2f}" for p, ms in sorted(row["mixed_phases_ms"].items())))
        rows.append(row)
        del t, o
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    for prec in ("f64", "mixed"):
        # slope of log(time) against log(N_k) between consecutive meshes
        for a, b in zip(rows[1:-1], rows[2:]):
            b[f"{prec}_exponent_from_prev"] = float(
                np.log(b[f"{prec}_ms"] / a[f"{prec}_ms"]) / np.log(b["N_k"] / a["N_k"]))
    print(json.dumps({"workload": "48-atom four-ring cell (60x75x54 grid, N 192, n_occ 84, "
                                  "N_ISDF 420) on 1^3..4^3 k-meshes", "series": rows}), flush=True)


def bench_ao_k(args):
    """THC-AO-K (Algorithm 1) as the composition of the stage-wise calls on the
    2x2x2 ring cell (N 192, n_occ 84, 60x75x54 grid): the AO-pair fit and its
    Coulomb matrices M^q once (exx_isdf_fit + exx_coulomb_V with the AO functions
    in place of the orbitals, N_ISDF = 2048 = 10.7 N, points by the GPU QRCP on
    the AO functions), then the per-iteration K-build from the occupied orbitals
    (exx_build_K), beside THC-oo-K's fused build of the same cell. FP64."""
    import torch

    import synth
    from paper_2304_05505_amd import exx
    from synth.fast import ao_on_grid_torch, orbitals_on_grid_torch

    dev = torch.device("cuda", 0)
    h = exx.Handle(0)
    cell = synth.make_config(2)
    N, nk, ng = cell.n_ao, cell.N_k, int(np.prod(cell.grid))
    ni = min(2048, 25 * N)
    phi = torch.stack([ao_on_grid_torch(cell, n, dev) for n in range(nk)]).contiguous()
    c_fit = exx.make_cell(cell.L, cell.grid, cell.kmesh, N, N, ni)
    pts = torch.empty((ni,), dtype=torch.int32, device=dev)
    npiv = torch.empty((1,), dtype=torch.int32, device=dev)
    t0 = time.perf_counter()
    exx.exx_select_points(h, c_fit, phi, pts, npiv)
    torch.cuda.synchronize()
    t_sel = time.perf_counter() - t0
    log(f"[ao-k] QRCP on the AO functions: {int(npiv.cpu()[0])} pivots in {t_sel:.1f} s")
    ao_pts = phi[:, :, pts.long()].permute(0, 2, 1).contiguous()  # (N_k, N_I, N)
    xi = torch.empty((nk, ni, ng), dtype=torch.complex128, device=dev)
    S = torch.empty((nk, ni, ni), dtype=torch.complex128, device=dev)
    V = torch.empty_like(S)
    rank = torch.empty((nk,), dtype=torch.int32, device=dev)

    def fit():
        exx.exx_isdf_fit(h, c_fit, exx.EXX_F64, phi, ao_pts, pts, xi, S, rank)
        exx.exx_coulomb_V(h, c_fit, exx.EXX_F64, xi, pts, V)

    s_fit = time_steps(fit, 1, 1, torch)
    log(f"[ao-k] AO-pair fit + M^q: {s_fit * 1e3:.1f} ms, ranks {rank.cpu().tolist()}")
    del xi, S
    torch.cuda.empty_cache()
    psi = orbitals_on_grid_torch(cell, synth.orbital_coeffs(cell), dev)
    occ = psi[:, :, pts.long()].permute(0, 2, 1).contiguous()
    c_k = exx.make_cell(cell.L, cell.grid, cell.kmesh, cell.n_occ, N, ni)
    o = outputs(torch, cell, dev)

    def iteration():
        exx.exx_build_K(h, c_k, exx.EXX_F64, ao_pts, occ, V, o["K"], o["Ex"])

    s_it = time_steps(iteration, max(1, args.steps), max(1, args.warmup), torch)
    ex_ao = float(o["Ex"].cpu()[0])
    log(f"[ao-k] per-iteration K-build: {s_it * 1e3:.2f} ms, E_x {ex_ao:.8f}")
    del V, phi, ao_pts
    torch.cuda.empty_cache()
    # THC-oo-K's fused build of the same cell (refit every iteration)
    t = cell_inputs(h, exx, torch, cell, dev)

    def oo():
        exx.exx_build(h, t["cell"], exx.EXX_F64, t["psi64"], t["occ_pts"], t["ao_pts"], t["pts"],
                      o["K"], o["Ex"], o["rank"])

    s_oo = time_steps(oo, max(1, args.steps), max(1, args.warmup), torch)
    ex_oo = float(o["Ex"].cpu()[0])
    log(f"[ao-k] THC-oo-K fused build: {s_oo * 1e3:.2f} ms, E_x {ex_oo:.8f}")
    del t
    torch.cuda.empty_cache()
    # THC-oo-K at the same point count as the AO fit: its least-squares fit
    # projects the occupied pairs, so |E_x| grows towards the exact value with
    # N_ISDF; the larger fit bounds how much exchange the exact answer holds
    from synth import cells as sc

    big = synth.make_ring_cell(sc.RING_CELL_L, sc.RING_CENTRES_4, cell.grid, cell.kmesh,
                               cell.n_occ, ni, (sc.SEED_ROOT, 2, 0), name="rings-k2-2048")
    t2 = cell_inputs(h, exx, torch, big, dev)
    exx.exx_build(h, t2["cell"], exx.EXX_F64, t2["psi64"], t2["occ_pts"], t2["ao_pts"], t2["pts"],
                  o["K"], o["Ex"], o["rank"])
    torch.cuda.synchronize()
    ex_oo_big = float(o["Ex"].cpu()[0])
    log(f"[ao-k] THC-oo-K with N_ISDF {ni}: E_x {ex_oo_big:.8f}")
    print(json.dumps({
        "workload": "48-atom four-ring cell, 2x2x2 k-mesh, N=192, n_occ=84, grid 60x75x54",
        "ao_k": {"n_isdf": ni, "n_pivot": int(npiv.cpu()[0]), "selection_s": t_sel,
                 "fit_and_Mq_ms": s_fit * 1e3, "per_iteration_ms": s_it * 1e3, "Ex": ex_ao},
        "oo_k": {"n_isdf": cell.n_isdf, "build_ms": s_oo * 1e3, "Ex": ex_oo,
                 "Ex_at_ao_k_point_count": ex_oo_big},
        "precision": "f64"}), flush=True)


def profile_target_ring(args, config):
    """A profiler's target for one ring cell: one untimed build per precision
    (F64, MIXED, F32), a marker dispatch (one-row exx_mlp_moments), one build per
    precision again (the measured ones), then a plain 1 GiB device copy whose
    counter readings calibrate the traffic counters."""
    import torch

    import synth
    from paper_2304_05505_amd import exx

    dev = torch.device("cuda", 0)
    h = exx.Handle(0)
    cell = synth.make_config(config)
    gold = load_json(f"config{config}.json")
    t = cell_inputs(h, exx, torch, cell, dev, pts=gold["pts"] if gold else None)
    o = outputs(torch, cell, dev)
    if args.potentials:
        # the exchange gradient and the robust-fit K instead of the builds
        from synth.fast import ao_on_grid_torch

        ao_grid = torch.stack([ao_on_grid_torch(cell, n, dev) for n in range(cell.N_k)])
        Kg = torch.empty_like(o["K"])
        for rep in range(2):
            if rep == 1:
                exx.exx_mlp_moments(h, torch.zeros((1, 3), dtype=torch.float32, device=dev),
                                    torch.zeros((6,), dtype=torch.float64, device=dev))
                torch.cuda.synchronize()
            exx.exx_exchange_gradient(h, t["cell"], t["psi64"], t["occ_pts"], t["ao_pts"], ao_grid,
                                      t["pts"], o["K"], Kg, o["Ex"], o["rank"])
            torch.cuda.synchronize()
            exx.exx_build_robust(h, t["cell"], t["psi64"], t["occ_pts"], t["ao_pts"], ao_grid,
                                 t["pts"], o["K"], o["Ex"], o["rank"])
            torch.cuda.synchronize()
            log(f"profile target: ring cell {config} potentials, pass {rep} done")
        return
    for rep in range(2):
        if rep == 1:
            exx.exx_mlp_moments(h, torch.zeros((1, 3), dtype=torch.float32, device=dev),
                                torch.zeros((6,), dtype=torch.float64, device=dev))
            torch.cuda.synchronize()
        for prec in ("f64", "mixed", "f32"):
            exx.exx_build(h, t["cell"], exx.PREC[prec], psi_for(t, prec, torch), t["occ_pts"],
                          t["ao_pts"], t["pts"], o["K"], o["Ex"], o["rank"])
            torch.cuda.synchronize()
        log(f"profile target: ring cell {config}, pass {rep} done")
    src = torch.ones((1 << 27,), dtype=torch.float64, device=dev)  # 1 GiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"profile target: copied {src.numel() * 8} bytes")


def profile_target(args):
    """The headline step for a profiler: the 24-cell batch in the mixed mode on
    concurrent lanes (after one untimed warm-up batch, which also tunes the tiles,
    and a one-row exx_mlp_moments dispatch that marks where the measured batch
    starts), then a plain 1 GiB device copy whose counter readings calibrate the
    traffic counters. With --phases the measured part is instead the pass of 24
    single MIXED builds with serial phase events from which the bench line's
    roofline is computed, and the phase times are printed."""
    import torch

    import synth
    from paper_2304_05505_amd import exx

    dev = torch.device("cuda", 0)
    h = exx.Handle(0)
    cells = synth.make_batch_cells()
    gold = load_json("config4.json")
    base = [cell_inputs(h, exx, torch, c, dev, pts=gold["cells"][i]["pts"] if gold else None)
            for i, c in enumerate(cells)]
    its = [dict(cell=t["cell"], psi_grid=psi_for(t, "mixed", torch), occ_pts=t["occ_pts"],
                ao_pts=t["ao_pts"], pts=t["pts"], **outputs(torch, c, dev))
           for c, t in zip(cells, base)]
    for rep in range(2):
        if rep == 1:
            # a marker dispatch between the tuning batch and the measured one
            exx.exx_mlp_moments(h, torch.zeros((1, 3), dtype=torch.float32, device=dev),
                                torch.zeros((6,), dtype=torch.float64, device=dev))
            torch.cuda.synchronize()
            if args.phases:
                break
        exx.exx_build_batched(h, its, exx.EXX_MIXED,
                              exx.EXX_BATCH_CONCURRENT | exx.EXX_BATCH_TUNE)
        torch.cuda.synchronize()
        log(f"profile target: mixed batch {rep} done")
    if args.phases:
        # the pass the bench line's roofline is measured on: every cell's build,
        # the normally overlapping phases one after another, with phase events
        h.set_timing(True, serial=True)
        phase_ms = {}
        for it in its:
            exx.exx_build(h, it["cell"], exx.EXX_MIXED, it["psi_grid"], it["occ_pts"],
                          it["ao_pts"], it["pts"], it["K"], it["Ex"], it["rank"])
            torch.cuda.synchronize()
            for p, (ms, _) in h.phase_times().items():
                phase_ms[p] = phase_ms.get(p, 0.0) + ms
        h.set_timing(False)
        log("profile target: phase pass done; phase ms " +
            ", ".join(f"{p} {ms:.2f}" for p, ms in sorted(phase_ms.items())))
    src = torch.ones((1 << 27,), dtype=torch.float64, device=dev)  # 1 GiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"profile target: copied {src.numel() * 8} bytes")


def run_records(out, workload, gold=None):
    """JSONL run records of one bench invocation: one record per measured path
    (config, dtype, E_x, |dE_x| and max|dK| against the stored oracle values,
    per-cell errors with the oracle's ranks and cond(S^m), time per phase and
    the phase rates)."""
    import datetime

    stamp = datetime.datetime.now(datetime.timezone.utc).isoformat(timespec="seconds")
    recs = []
    if workload == "batch24":
        cells = gold["cells"] if gold else None
        for prec, r in out.get("batched", {}).items():
            per = out.get("batched_per_cell", {}).get(prec, {})
            rec = {"time": stamp, "workload": "batch24", "path": f"batched-{prec}", "dtype": prec,
                   "ms_per_step": r.get("seconds", 0.0) * 1e3,
                   "builds_per_s": r.get("builds_per_s"),
                   "max_dEx": r.get("max_dEx_vs_oracle"), "max_dK": r.get("max_dK_vs_oracle"),
                   "cells_in_gate": r.get("cells_meeting_gate")}
            if cells and per.get("dEx") is not None:
                rec["cells"] = [{"name": c["name"], "Ex_oracle": c["Ex"], "dEx": dE, "max_dK": dK,
                                 "rank": c["rank"], "cond_S_max": max(c["cond_S"])}
                                for c, dE, dK in zip(cells, per["dEx"], per["dK"])]
            if prec == out.get("config", {}).get("prec"):
                rec["phases_ms"] = out.get("phases_ms_batch_mixed")
                rec["phase_rates"] = out.get("phase_rates_batch_mixed")
                rec["roofline"] = out.get("roofline")
            recs.append(rec)
    for leg_name, leg in out.get("paths", {}).items():
        for label, r in leg.get("paths", {}).items():
            recs.append({"time": stamp, "workload": leg_name, "path": label,
                         "dtype": r.get("precision"),
                         "ms": r.get("ms_per_build", r.get("ms_per_call")), "Ex": r.get("Ex"),
                         "dEx": r.get("dEx_vs_oracle"), "max_dK": r.get("maxdK_vs_oracle"),
                         "phases_ms": r.get("phases_ms")})
    return recs


def write_records(path, recs):
    with open(path, "a") as f:
        for r in recs:
            f.write(json.dumps(r) + "\n")
    log(f"appended {len(recs)} run records to {path}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--record", metavar="PATH",
                    help="append JSONL run records (one per measured path) to PATH")
    ap.add_argument("--profile", action="store_true")
    ap.add_argument("--phases", action="store_true",
                    help="with --profile on the batch: after the tuning batch, profile the "
                         "pass of single builds with phase events that the roofline uses")
    ap.add_argument("--potentials", action="store_true",
                    help="with --profile and a ring workload: profile the exchange gradient "
                         "and the robust-fit K instead of the builds")
    ap.add_argument("--workload", choices=("batch24", "rings-k2", "rings-k3", "select-k4",
                                            "nk-series", "ao-k"), default="batch24")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (got --gpus {args.gpus}); across GPUs the batch would "
              "shard by cell with no exchange, which is not timed", file=sys.stderr)
        sys.exit(2)
    if args.workload == "select-k4":
        bench_select5(args)
        return
    if args.workload == "nk-series":
        bench_nk_series(args)
        return
    if args.workload == "ao-k":
        bench_ao_k(args)
        return
    if args.profile:
        if args.workload in ("rings-k2", "rings-k3"):
            profile_target_ring(args, 2 if args.workload == "rings-k2" else 3)
        else:
            profile_target(args)
        return

    import torch

    from paper_2304_05505_amd import exx

    dev = torch.device("cuda", 0)
    h = exx.Handle(0)
    if args.workload in ("rings-k2", "rings-k3"):
        leg = ring_leg(2 if args.workload == "rings-k2" else 3, args, h, exx, torch, dev)
        print(json.dumps(leg), flush=True)
        if args.record:
            write_records(args.record, run_records({"paths": {args.workload: leg}},
                                                   args.workload))
        return

    cells, res, seq_r, phase_ms, wex, wsv, units = batch_leg(args, h, exx, torch, dev)
    legs = {}
    for cfg in (3, 2):
        legs[f"rings-k{cfg}"] = ring_leg(cfg, args, h, exx, torch, dev)
    ok = [p for p in ("mixed", "f32", "f64")
          if res[p].get("cells_meeting_gate", 0) == 24]
    chosen = "mixed"
    r = res[chosen]
    roof = roofline(phase_ms, wex, wsv, units, chosen)
    roof["kernel"] = KERNELS.get(roof["phase"], ("?", "?"))
    out = {
        "metric": METRIC,
        "value": r["builds_per_s"],
        "unit": "K-builds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["seconds"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {
            "workload": "24-cell batch: 2 x {8, 16, 24, 48 atoms} x {1^3, 2^3, 3^3} k-meshes, 4 "
                        "Gaussian functions/atom (N 32-192), n_occ = 0.44 N, N_ISDF = 2.2 N, grids "
                        "4.5 points/bohr; one exx_build_batched call per step (captured graph or "
                        "concurrent lanes, the faster), mixed mode",
            "batch_mode": r["mode"],
            "cells": 24,
            "prec": chosen,
        },
        "speedup_vs_sequential_f64": r["speedup_vs_sequential_f64"],
        "sequential_f64": seq_r,
        "meets_gate": bool(chosen in ok),
        "gate": {"dEx_Ha_per_cell": GATE_E, "max_dK": GATE_K, "vs": "stored FP64 oracle values"},
        "settings": {"refinement_steps": 0, "contraction": "FP64 matrix cores",
                     "fit": "one per transfer"},
        "roofline": roof,
        "batched": {p: {k: v for k, v in res[p].items() if not k.endswith("per_cell")}
                    for p in res},
        "batched_per_cell": {p: {"dEx": res[p].get("dEx_per_cell"), "dK": res[p].get("dK_per_cell")}
                             for p in res},
        "phases_ms_batch_mixed": phase_ms,
        "phase_rates_batch_mixed": {p: phase_rate(p, phase_ms, wex, wsv, units, chosen)
                                    for p in wex if phase_ms.get(p, 0) > 0},
        "paths": legs,
    }
    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(cells)
    print(json.dumps(out), flush=True)
    if args.record:
        write_records(args.record, run_records(out, "batch24", load_json("config4.json")))


if __name__ == "__main__":
    main()
