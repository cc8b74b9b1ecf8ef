"""Throughput of the THC-oo-K exchange build (K^k for all k plus E_x) on one GPU.

Workload: the 48-atom four-ring cell (14.0 x 17.8 x 12.9 bohr, C6H6 x 4) on a
2x2x2 Gamma-centred k-mesh; s + p Gaussians per atom (N = 192), n_occ = 84,
grid 60x75x54 (N_g = 243000), N_ISDF = 420 points chosen on the GPU by
pivoted-Cholesky QRCP. Seeded synthetic orbitals; inputs are resident in HBM
before the timed region. One step = one whole K-build (fit, Coulomb
matrices, contraction) through the C ABI.

Three precision paths are timed: f64 (everything FP64), mixed (FP64 fit,
FP32 FFT and Coulomb contraction with FP64 accumulation) and f32 (bulk FP32).
`value` is the fastest path whose E_x and K stay within 1e-5 Ha/cell and
1e-6 of the FP64 result (the FP64 path itself matches the FP64 oracle to
~1e-12; with --prec the reported path is forced).

Prints one JSON line. Options: --steps K --warmup W --gpus N (N must be 1)
--prec auto|f64|mixed|f32 --no-cpu --profile; --workload select-k4 instead times
the learned and the QRCP point selection at the 4x4x4 ring workload, each
followed by one FP32 K-build; --workload batch24 times the 24-cell batched
build (one graph launch) against 24 sequential FP64 builds.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "K-builds/sec (all k) vs plain FP64 GPU at |ΔE_x|≤1e-5 Ha/cell; MFMA %"
PEAK = {  # MI355X published dense peaks
    "hbm_GBs": 8000.0,
    "fp64_TF": 78.6,
    "fp32_TF": 157.3,
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def real_path(cell):
    """The fused build's real path runs on meshes whose every axis has N_i <= 2."""
    return all(n <= 2 for n in cell.kmesh)


def algorithmic_work(cell, n_isdf, prec):
    """Per-launch algorithmic flops / bytes of each phase (one K-build).

    Flops count the real multiply-adds of the product form each kernel uses:
    complex products on the FP64 matrix cores use Gauss's three-product form, 6
    flops per complex multiply-add; the FP32-matrix-core Gamma of the FP32 path
    and the small K GEMMs use four real products, 8 flops. The Coulomb
    contraction forms the lower triangle only (N_ISDF^2/2 pairs).
    On the real path (every k-mesh axis <= 2) the solve is a real GEMM (2 flops
    per multiply-add), Z~ and eta are real arrays, the FFT writes the kept half
    grid of n1 n2 (n3/2 + 1) points and the Coulomb contraction takes
    Re(X conj Y) (two real products, 4 flops) over that half grid; in FP32 the
    Gamma GEMM and the k-correlation are one kernel (phase "gamma"). There the
    solve multiplies by the triangular inverse Cholesky factor and counts its
    N_I (N_I + 1) / 2 multiply-adds per grid point (the kernel rounds each
    16-row block up to the diagonal).
    """
    nk, ng, no, na = cell.N_k, cell.N_g, cell.n_occ, cell.n_ao
    ni = n_isdf
    cs = 16 if prec == "f64" else 8           # complex Gamma/Z (f64, mixed: Gamma c128)
    cg = 8.0 if prec == "f32" else 6.0        # flops per complex multiply-add of the Gamma GEMM
    work = {"gamma": ("flop", cg * nk * ni * no * ng),
            "K": ("flop", 8.0 * nk * (na * ni * ni + na * na * ni))}
    if real_path(cell):
        n1, n2, n3 = cell.grid
        if prec == "f32":
            # FP32: one fused kernel forms Gamma^n (four real products) and Z~;
            # its time is reported under "gamma" and counts the GEMM flops
            work["gamma"] = ("flop", 8.0 * nk * ni * no * ng)
        ngh = n1 * n2 * (n3 // 2 + 1)
        gam = 8 if prec == "f32" else 16      # Gamma element (complex)
        zr = 4 if prec == "f32" else 8        # Z~ element (real)
        xr = 8 if prec == "f64" else 4        # eta element (real)
        xc = 16 if prec == "f64" else 8       # transform element (complex)
        work.update({
            "kcorr": ("byte", nk * ni * ng * (gam + zr)),
            # the lower-triangular inverse factor W (S~^+ = W^T W): N_I (N_I + 1) / 2
            # multiply-adds per grid point
            "solve": ("flop", 1.0 * ni * (ni + 1) * nk * ng),
            "fft": ("byte", nk * ni * (ng * xr + ngh * xc)),
            "coulomb": ("flop", 2.0 * nk * ni * ni * ngh),
        })
    else:
        work.update({
            "kcorr": ("byte", 2.0 * nk * ni * ng * cs),
            "solve": ("flop", 6.0 * nk * ni * ni * ng),
            "fft": ("byte", 2.0 * nk * ni * ng * cs),
            "coulomb": ("flop", 3.0 * nk * ni * ni * ng),
        })
    return work


# HBM traffic of the dominant kernel of each phase at this workload, from two
# rocprofv3 counter runs of `bench.py --profile` (FETCH_SIZE, then WRITE_SIZE; KiB
# per dispatch; the FP64 transform and contraction run in four chunks of transfers,
# so their entries cover a quarter of the build). A plain 1 GiB device copy reads
# 524 312 KiB of FETCH_SIZE and 1 048 576 KiB of WRITE_SIZE on MI355X, so fetch
# counts are scaled by 2.0 and write counts by 1.0. Each entry names the source file of its kernels and that file's
# SHA-256 prefix when the counters were taken; a changed file reports null.
FETCH_SCALE, WRITE_SCALE = 1048576.0 / 524312.2, 1.0
TRAFFIC = {
    # (phase, path): (source, sha256[:16], FETCH_SIZE KiB, WRITE_SIZE KiB)
    ("solve", "f64"): ("gemm_mfma.hip", "b285ff3ab7358f19", 8087716.2, 6469594.8),
    ("solve", "mixed"): ("gemm_mfma.hip", "b285ff3ab7358f19", 7483829.7, 3303541.6),
    ("solve", "f32"): ("gemm_mfma.hip", "b285ff3ab7358f19", 3051883.4, 3263706.8),
    ("gamma", "f64"): ("gemm_mfma.hip", "b285ff3ab7358f19", 1299417.4, 12757500.0),
    ("gamma", "mixed"): ("gemm_mfma.hip", "b285ff3ab7358f19", 1299417.4, 12757500.0),
    ("gamma", "f32"): ("fit.hip", "fa8c9af02b7f561a", 1355649.1, 4503349.7),
    ("kcorr", "f64"): ("fit.hip", "fa8c9af02b7f561a", 6378788.6, 6378750.0),
    ("kcorr", "mixed"): ("fit.hip", "fa8c9af02b7f561a", 6378788.6, 6378750.0),
    ("fft", "f64"): ("fft.hip", "05376b4f2156bb5c", 1835594.0, 3307500.8),
    ("fft", "mixed"): ("fft.hip", "05376b4f2156bb5c", 3884780.6, 6615000.5),
    ("fft", "f32"): ("fft.hip", "05376b4f2156bb5c", 3884780.6, 6615000.5),
    ("coulomb", "f64"): ("coulomb.hip", "e5d3729797beb400", 4980022.1, 210761.8),
    ("coulomb", "mixed"): ("coulomb.hip", "e5d3729797beb400", 8965173.4, 206327.3),
    ("coulomb", "f32"): ("coulomb.hip", "e5d3729797beb400", 8965173.4, 206327.3),
}


def traffic_bytes(phase, path):
    """HBM bytes per launch of the phase's kernel, or None if unmeasured or changed."""
    import hashlib

    ent = TRAFFIC.get((phase, path))
    if ent is None:
        return None
    src, digest, fetch_kib, write_kib = ent
    fn = os.path.join(ROOT, "paper_2304_05505_amd", "csrc", src)
    try:
        cur = hashlib.sha256(open(fn, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    if cur != digest:
        return None
    return 1024.0 * (fetch_kib * FETCH_SCALE + write_kib * WRITE_SCALE)


FP64_PHASES = {"f64": {"gamma", "solve", "coulomb", "K"},
               "mixed": {"gamma", "solve", "coulomb", "K"},
               "f32": {"solve", "coulomb", "K"}}


def roofline(phases, work, prec, steps):
    """Roofline entry for the phase with the largest time."""
    best = max((p for p in phases if p in work), key=lambda p: phases[p][0])
    ms, calls = phases[best]
    avg_s = ms / steps / 1e3  # per build (a phase may run as several launches per build)
    kind, amount = work[best]
    traffic = traffic_bytes(best, prec)
    if kind == "byte":
        achieved = amount / avg_s / 1e9
        return best, {"bound": "hbm", "achieved": achieved, "peak": PEAK["hbm_GBs"], "unit": "GB/s",
                      "frac": achieved / PEAK["hbm_GBs"], "traffic": traffic}
    achieved = amount / avg_s / 1e12
    peak = PEAK["fp64_TF"] if best in FP64_PHASES[prec] else PEAK["fp32_TF"]
    return best, {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                  "frac": achieved / peak, "traffic": traffic}


def cpu_baseline(cell, psi, pts, ao):
    """The FP64 oracle on a bounded sample: all Gamma^n plus the fit/FFT/Coulomb of two q."""
    from oracle import thc
    from oracle._threads import WORKERS

    t0 = time.perf_counter()
    o = thc.thc_oo_k(cell.L, cell.grid, cell.kmesh, psi, pts, ao,
                     m_subset=[cell.N_k - 1, cell.N_k // 2])
    wall = time.perf_counter() - t0
    sec = o["seconds"]
    est = sec["gamma"] + cell.N_k * float(np.mean(sec["per_q"])) + sec["contract"]
    return {
        "value": 1.0 / est,
        "unit": "K-builds/s",
        "cores": WORKERS,
        "kind": "oracle",
        "sample": (f"oracle Gamma^n for all {cell.N_k} k plus steps 2-6 for two of {cell.N_k} "
                   f"transfers ({wall:.1f} s wall); build time extrapolated as "
                   f"gamma + N_k * per_q + contract = {est:.1f} s"),
    }


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

    def learned():
        pts = torch.empty((ni,), dtype=torch.int32, device=dev)
        used, resid = exx.exx_select_points_mlp(h, c, psi64, w["norm"], theta, w["tau"],
                                                int(w["n_probe"]), pts)
        return pts, used, resid

    learned()
    (pm, used, resid), t_mlp = timed(learned, 3)
    log(f"[select5] learned selection {t_mlp * 1e3:.1f} ms (fallback {used}, residual {resid:.4f})")
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
    log(f"[select5] K-build (f32) at learned points {tb_m * 1e3:.1f} ms, E_x {ex_m:.8f}")
    ex_q, tb_q = build(pq)
    log(f"[select5] K-build (f32) at QRCP points {tb_q * 1e3:.1f} ms, E_x {ex_q:.8f}")
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
        "learned": {"select_s": t_mlp, "build_s": tb_m, "Ex": ex_m, "probe_residual": resid,
                    "fallback": used},
        "qrcp": {"select_s": t_qrcp, "build_s": tb_q, "Ex": ex_q, "probe_residual": resid_q},
        "end_to_end_speedup": (t_qrcp + tb_q) / (t_mlp + tb_m),
        "dEx_learned_vs_qrcp": ex_m - ex_q,
    }
    print(json.dumps(out), flush=True)


def bench_batch24(args):
    """The 24-cell batch (2 x {8, 16, 24, 48 atoms} x {1, 2, 3}^3 k-meshes): one
    batched call (hipGraph replay, autotuned tiles) against 24 sequential plain
    FP64 builds, with the per-cell E_x and K differences."""
    import torch

    import synth
    from paper_2304_05505_amd import exx
    from synth.fast import orbitals_on_grid_torch

    dev = torch.device("cuda", 0)
    h = exx.Handle(0)
    t0 = time.perf_counter()
    items64, items_mx, items32 = [], [], []
    for cell in synth.make_batch_cells():
        psi = orbitals_on_grid_torch(cell, synth.orbital_coeffs(cell), dev)
        c = exx.make_cell(cell.L, cell.grid, cell.kmesh, cell.n_occ, cell.n_ao, cell.n_isdf)
        pts_t = torch.empty((cell.n_isdf,), dtype=torch.int32, device=dev)
        npiv = torch.empty((1,), dtype=torch.int32, device=dev)
        exx.exx_select_points(h, c, psi, pts_t, npiv)
        pts = pts_t.cpu().numpy().astype(np.int64)
        ao = np.stack([synth.ao_at_points(cell, n, pts) for n in range(cell.N_k)])
        t_ao = torch.from_numpy(np.ascontiguousarray(np.transpose(ao, (0, 2, 1)))).to(dev)
        occ = psi[:, :, pts_t.long()].permute(0, 2, 1).contiguous()
        base = {"cell": c, "occ_pts": occ, "ao_pts": t_ao, "pts": pts_t}
        for lst, p in ((items64, psi), (items_mx, psi), (items32, psi.to(torch.complex64))):
            lst.append(dict(base, psi_grid=p,
                            K=torch.empty((cell.N_k, cell.n_ao, cell.n_ao), dtype=torch.complex128,
                                          device=dev),
                            Ex=torch.empty((1,), dtype=torch.float64, device=dev),
                            rank=torch.empty((cell.N_k,), dtype=torch.int32, device=dev)))
    torch.cuda.synchronize()
    log(f"[batch24] inputs and QRCP points for 24 cells in {time.perf_counter() - t0:.1f} s")

    def sequential_f64():
        for it in items64:
            exx.exx_build(h, it["cell"], exx.EXX_F64, it["psi_grid"], it["occ_pts"], it["ao_pts"],
                          it["pts"], it["K"], it["Ex"], it["rank"])

    stream = torch.cuda.Stream()

    def batched(prec, items):
        stream.wait_stream(torch.cuda.current_stream())
        exx.exx_build_batched(h, items, prec, exx.EXX_BATCH_GRAPH | exx.EXX_BATCH_TUNE,
                              stream=stream)
        stream.synchronize()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts))

    reps = max(1, min(args.steps, 3))
    t_seq = timed(sequential_f64, reps)
    ex64 = [float(it["Ex"].cpu()[0]) for it in items64]
    k64 = [it["K"].cpu().numpy() for it in items64]
    log(f"[batch24] 24 sequential FP64 builds: {t_seq * 1e3:.1f} ms")
    res = {}
    for name, prec, items in (("f32", exx.EXX_F32, items32), ("mixed", exx.EXX_MIXED, items_mx),
                              ("f64", exx.EXX_F64, items64)):
        t_b = timed(lambda: batched(prec, items), reps)
        dEs = [abs(float(it["Ex"].cpu()[0]) - e) for it, e in zip(items, ex64)]
        dKs = [float(np.abs(it["K"].cpu().numpy() - k).max()) for it, k in zip(items, k64)]
        dE, dK = max(dEs), max(dKs)
        res[name] = {"seconds": t_b, "builds_per_s": 24.0 / t_b, "speedup_vs_seq_f64": t_seq / t_b,
                     "max_dEx_vs_f64": dE, "max_dK_vs_f64": dK,
                     "meets_1e-5_1e-6": bool(dE <= 1e-5 and dK <= 1e-6),
                     "dEx_per_cell": dEs, "dK_per_cell": dKs,
                     "maxabs_K_per_cell": [float(np.abs(k).max()) for k in k64]}
        log(f"[batch24] batched {name}: {t_b * 1e3:.1f} ms, max|dEx| {dE:.2e}, max|dK| {dK:.2e}")
    ok = [n for n in res if res[n]["meets_1e-5_1e-6"]]
    chosen = max(ok, key=lambda n: res[n]["builds_per_s"])
    out = {
        "metric": "K-builds/s over a 24-cell batch (one graph launch) vs 24 sequential plain FP64 "
                  "builds, at |dE_x| <= 1e-5 Ha/cell and max|dK| <= 1e-6",
        "value": res[chosen]["builds_per_s"],
        "path": chosen,
        "unit": "K-builds/s",
        "n_gpus": 1,
        "steps": reps,
        "higher_is_better": True,
        "vs_baseline": None,
        "dtype": {"f64": "f64", "mixed": "f64+f32", "f32": "f32+f64"}[chosen],
        "data": "synthetic",
        "config": {"workload": "24 cells: 2 x {8, 16, 24, 48 atoms} x {1, 2, 3}^3 k-meshes, 4 "
                               "functions/atom, n_occ = 0.44 N, N_ISDF = 2.2 N, QRCP points"},
        "sequential_f64_s": t_seq,
        "batched": res,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", choices=("auto", "f64", "mixed", "f32"), default="auto")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="profiling target: one build per precision path and a 1 GiB device "
                         "copy, no JSON")
    ap.add_argument("--workload", choices=("rings-k2", "select-k4", "batch24"), default="rings-k2",
                    help="rings-k2: the K-build throughput line (default); select-k4: learned vs "
                         "QRCP selection + K-build at the 4x4x4 ring workload; batch24: the "
                         "24-cell batched build against sequential FP64 builds")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the build is not sharded "
              "across GPUs", file=sys.stderr)
        sys.exit(2)
    if args.workload == "select-k4":
        bench_select5(args)
        return
    if args.workload == "batch24":
        bench_batch24(args)
        return

    import torch

    import synth
    from paper_2304_05505_amd import exx

    dev = torch.device("cuda", 0)
    cell = synth.make_config(2)
    t0 = time.perf_counter()
    C = synth.orbital_coeffs(cell)
    psi = synth.orbitals_on_grid(cell, C)
    log(f"inputs generated in {time.perf_counter() - t0:.1f} s")
    nk, no, ng, ni, na = cell.N_k, cell.n_occ, cell.N_g, cell.n_isdf, cell.n_ao

    h = exx.Handle(0)
    c = exx.make_cell(cell.L, cell.grid, cell.kmesh, no, na, ni)
    t_psi64 = torch.from_numpy(psi).to(dev)
    t_pts = torch.empty((ni,), dtype=torch.int32, device=dev)
    t_npiv = torch.empty((1,), dtype=torch.int32, device=dev)
    t0 = time.perf_counter()
    exx.exx_select_points(h, c, t_psi64, t_pts, t_npiv)
    torch.cuda.synchronize()
    log(f"points selected on the GPU in {time.perf_counter() - t0:.2f} s")
    pts = t_pts.cpu().numpy().astype(np.int64)
    ao = np.stack([synth.ao_at_points(cell, n, pts) for n in range(nk)])
    t_ao = torch.from_numpy(np.ascontiguousarray(np.transpose(ao, (0, 2, 1)))).to(dev)
    t_occ = torch.from_numpy(np.ascontiguousarray(np.transpose(psi[:, :, pts], (0, 2, 1)))).to(dev)
    t_psi32 = t_psi64.to(torch.complex64)

    if args.profile:
        # one build per precision path, then a plain 1 GiB device copy whose
        # counter readings calibrate the HBM traffic counters
        K = torch.empty((nk, na, na), dtype=torch.complex128, device=dev)
        Ex = torch.empty((1,), dtype=torch.float64, device=dev)
        rank = torch.empty((nk,), dtype=torch.int32, device=dev)
        for prec in ("f64", "mixed", "f32"):
            t_psi = t_psi32 if prec == "f32" else t_psi64
            exx.exx_build(h, c, exx.PREC[prec], t_psi, t_occ, t_ao, t_pts, K, Ex, rank)
            torch.cuda.synchronize()
            log(f"profile target [{prec}] done: Ex {float(Ex.cpu()[0]):.12f}")
        src = torch.ones((1 << 27,), dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"profile target: copied {src.numel() * 8} bytes")
        return

    results = {}
    for prec in ("f64", "mixed", "f32"):
        p = exx.PREC[prec]
        t_psi = t_psi32 if prec == "f32" else t_psi64
        K = torch.empty((nk, na, na), dtype=torch.complex128, device=dev)
        Ex = torch.empty((1,), dtype=torch.float64, device=dev)
        rank = torch.empty((nk,), dtype=torch.int32, device=dev)

        def step():
            exx.exx_build(h, c, p, t_psi, t_occ, t_ao, t_pts, K, Ex, rank)

        # per-phase HIP events on the build's stream, recorded inside the timed
        # region; the warmup steps fill the handle's event pool
        h.set_timing(True)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        h.phase_times()
        log(f"[{prec}] warmup done")
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        phases = h.phase_times()
        h.set_timing(False)
        log(f"[{prec}] {args.steps} steps in {el:.3f} s; phases(ms/build): " +
            ", ".join(f"{k}={v[0] / args.steps:.2f}" for k, v in phases.items()))
        results[prec] = {
            "value": args.steps / el,
            "ms_per_step": el / args.steps * 1e3,
            "Ex": float(Ex.cpu()[0]),
            "K": K.cpu().numpy(),
            "rank": rank.cpu().tolist(),
            "phases": phases,
        }

    ref64 = results["f64"]
    gold = None
    gpath = os.path.join(ROOT, "tests", "golden", "config2.json")
    if os.path.exists(gpath):
        g = json.load(open(gpath))
        if g["pts"] == [int(x) for x in pts]:
            gold = g
    paths = {}
    for prec, r in results.items():
        dE = abs(r["Ex"] - ref64["Ex"])
        dK = float(np.abs(r["K"] - ref64["K"]).max())
        paths[prec] = {"value": r["value"], "ms_per_step": r["ms_per_step"], "Ex": r["Ex"],
                       "dEx_vs_f64": dE, "maxdK_vs_f64": dK,
                       "speedup_vs_f64": r["value"] / ref64["value"],
                       "meets_1e-5_1e-6": bool(dE <= 1e-5 and dK <= 1e-6)}
        if gold is not None:
            paths[prec]["dEx_vs_oracle"] = abs(r["Ex"] - gold["Ex"])
    if args.prec == "auto":
        ok = [p for p in paths if paths[p]["meets_1e-5_1e-6"]]
        chosen = max(ok, key=lambda p: paths[p]["value"])
    else:
        chosen = args.prec
    sel = results[chosen]
    work = algorithmic_work(cell, ni, "f64" if chosen == "f64" else "f32")
    dom, roof = roofline(sel["phases"], work, chosen, args.steps)
    out = {
        "metric": METRIC,
        "value": sel["value"],
        "unit": "K-builds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sel["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "mixed": "f64+f32", "f32": "f32+f64"}[chosen],
        "data": "synthetic",
        "config": {
            "workload": "THC-oo-K K-build, 48-atom four-ring cell, 2x2x2 k-mesh, N=192, n_occ=84, "
                        "grid 60x75x54, N_ISDF=420",
            "N_k": nk, "N_g": ng, "n_occ": no, "n_ao": na, "n_isdf": ni,
            "prec": chosen,
        },
        "roofline": dict(roof, kernel=dom),
        "paths": paths,
        "oracle_points": gold is not None,
        "phases_ms": {k: v[0] / args.steps for k, v in sel["phases"].items()},
    }
    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(cell, psi, pts, ao)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
