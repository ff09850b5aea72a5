#!/usr/bin/env python3
"""Benchmark: time-to-solution of bootstrapped block Lanczos on one MI355X.

Workload (synthetic, seeded): n = 2,000,000, ~200 nnz/row (4.0e8 nnz), 2000
sectors of 1000 rows, 70/30 in-sector/partner split; FP32 values with int32
columns; block size 8, lowest 10 eigenpairs to residual 1e-6 * ||H||; pivot
bootstrapped from the leading 20,000-row block.  One step = bootstrap pivot +
block Lanczos to convergence + Ritz vectors + explicit FP64 residual, with the
matrix already resident in HBM.

Prints ONE JSON line (metric, value = mean time-to-solution in seconds, ...)
with a "roofline" object for the CSR SpMM (its launches inside the timed
solves, each bracketed by HIP events that the library records on the solver's
stream) and a "cpu_baseline" object (the FP64 CPU oracle timed on a bounded
sample of the same solve on the host cores).

--compare-pivots solves the held-out n = 5e6 instance (~300 nnz/row, b = k = 10,
tol 1e-6, truncation 50,000 rows) from four pivots -- random, bootstrapped,
the one-hop Rayleigh-Ritz block P_D alone, and the learned proposer with its
fallback -- and prints one JSON line with the counts and times of each.

Two helper modes serve the hardware-counter measurement of HBM traffic:
  --kernels-only       runs the SpMM, the reorthogonalisation gram and a plain
                       1 GiB elementwise copy a few times each (the program run
                       under `rocprofv3 --pmc FETCH_SIZE` and `--pmc WRITE_SIZE`);
  --traffic F W        reads the two counter CSV directories and writes the
                       per-launch HBM bytes of the SpMM, scaled by what the
                       same counters read for the copy, to
                       profiles/spmm_mid_n2e6_traffic.json.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

# the CPU baseline's OpenMP threads stay close to each other (set before any
# OpenMP runtime starts)
os.environ.setdefault("OMP_PROC_BIND", "close")

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # B/s, MI355X HBM3E
FP64_PEAK = 78.6e12        # FLOP/s, MI355X FP64 (vector and matrix)
WORKLOAD = "mid_n2e6"


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def load_matrix(w):
    import synthgen
    cache = os.environ.get("BBL_CACHE_DIR")
    key = "%s_%d_%d_%d_%g_%d" % (w.name, w.n, w.R, w.q, w.p, w.seed)
    if cache:
        os.makedirs(cache, exist_ok=True)
        base = os.path.join(cache, key)
        if os.path.exists(base + ".val.npy"):
            H = synthgen.CSR(w.n, np.load(base + ".rp.npy"), np.load(base + ".col.npy"),
                             np.load(base + ".val.npy"), None, None, w.R)
            return H
    H = w.generate()
    if cache:
        np.save(base + ".rp.npy", H.row_ptr)
        np.save(base + ".col.npy", H.col)
        np.save(base + ".val.npy", H.val)
    return H


def spmm_bytes(n, nnz, b, sv, sx):
    # values + columns streamed once, row pointers, V read once, W written once
    return nnz * (sv + 4) + 8 * (n + 1) + 2 * n * b * sx


def solve_bytes(n, nnz, b, k, iters, extra_spmm, second_passes):
    """HBM bytes the phases of one block Lanczos solve move at least (FP32
    matrix values and basis, FP64 W' and Ritz vectors), block by block:
    SpMM; A_j gram (V_j and W); three-term update (W, V_{j-1:j} in, W' out);
    Gram-Schmidt gram and update over the j + 1 stored blocks (W' read, and
    read and written); Cholesky QR (W' read and written, then read, V_{j+1}
    written).  Then the Ritz vectors (basis read, X written, normalised in
    place) and the FP64 residual (matrix once, X read twice), plus the
    second Gram-Schmidt sweeps and any SpMM calls beyond one per block."""
    blk = n * b * 4      # one FP32 basis block
    wp = n * b * 8       # W' in FP64
    sp = spmm_bytes(n, nnz, b, 4, 4)
    tot = 0.0
    for j in range(iters):
        tot += sp + 2 * blk + (blk + min(j + 1, 2) * blk + wp)
        tot += ((j + 1) * blk + wp) + ((j + 1) * blk + 2 * wp)
        tot += 3 * wp + blk
    jm = iters / 2.0
    tot += second_passes * (2 * (jm + 1) * blk + 3 * wp)
    tot += extra_spmm * sp
    tot += iters * blk + n * k * 8 + 2 * n * k * 8
    tot += nnz * 8 + 8 * (n + 1) + 2 * n * k * 8
    return tot


def source_hash(*names):
    h = hashlib.sha256()
    for nm in names:
        with open(os.path.join(ROOT, "paper_2210_15763_amd", "csrc", nm), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(kernel_hash):
    """HBM bytes per SpMM launch measured with rocprofv3 counters (committed
    summary), or None when the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", "spmm_mid_n2e6_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("spmm_source_hash") != kernel_hash:
        return None
    return rec.get("hbm_bytes_per_launch")


COPY_BYTES = 1 << 30   # bytes read (and written) by the calibration copy


def _counter_rows(d):
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            rows.extend(csv.DictReader(fh))
    if not rows:
        raise SystemExit("no counter_collection.csv under " + d)
    return rows


def _per_dispatch(rows, counter, match):
    """Mean over dispatches of kernels whose name contains `match` of the
    counter (summed over its instances within one dispatch)."""
    per = {}
    for r in rows:
        if r.get("Counter_Name") != counter or match not in r.get("Kernel_Name", ""):
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    if not per:
        raise SystemExit("no %s rows for kernels matching %r" % (counter, match))
    return float(np.mean(list(per.values()))), len(per)


SPMM_PASSES = ("k_spmm_pipe12<8, false, float>", "k_spmm_rest<8, false, float>")
REORTH_BLOCKS = 50   # basis blocks of the counter runs' gram and update


def write_traffic(fetch_dir, write_dir):
    """FETCH_SIZE and WRITE_SIZE are in KiB per dispatch; each is scaled by
    the ratio of known bytes to the counter's reading for the copy kernel.  One
    planned SpMM is two dispatches (passes 1-2 fused, pass 3): their means are added."""
    fr, wr_ = _counter_rows(fetch_dir), _counter_rows(write_dir)
    fp = [_per_dispatch(fr, "FETCH_SIZE", k) for k in SPMM_PASSES]
    wp = [_per_dispatch(wr_, "WRITE_SIZE", k) for k in SPMM_PASSES]
    f_spmm, nf = sum(x[0] for x in fp), [x[1] for x in fp]
    w_spmm, nw = sum(x[0] for x in wp), [x[1] for x in wp]
    f_copy, _ = _per_dispatch(_counter_rows(fetch_dir), "FETCH_SIZE", "neg")
    w_copy, _ = _per_dispatch(_counter_rows(write_dir), "WRITE_SIZE", "neg")
    fetch_scale = COPY_BYTES / (f_copy * 1024.0)
    write_scale = COPY_BYTES / (w_copy * 1024.0)
    rd = f_spmm * 1024.0 * fetch_scale
    wr = w_spmm * 1024.0 * write_scale
    import synthgen
    w = synthgen.WORKLOADS[WORKLOAD]
    H = load_matrix(w)
    alg = spmm_bytes(H.n, H.nnz, w.nvec, 4, 4)
    rec = {"kernel": "k_spmm_pipe12<8, false, float> + k_spmm_rest<8, false, float> (one planned SpMM: passes 1 and 2 in "
                     "one kernel, then pass 3; float32 values and vectors, 8 vectors, sectors "
                     "of 1000 rows, two sets of column blocks staged in LDS, the rest gathered)",
           "workload": WORKLOAD, "per_pass_fetch_kib": [x[0] for x in fp],
           "per_pass_write_kib": [x[0] for x in wp],
           "spmm_source_hash": source_hash("spmm.hip"),
           "fetch_kib_per_launch": f_spmm, "write_kib_per_launch": w_spmm,
           "copy_fetch_kib": f_copy, "copy_write_kib": w_copy,
           "fetch_scale": fetch_scale, "write_scale": write_scale,
           "hbm_read_bytes_per_launch": rd, "hbm_write_bytes_per_launch": wr,
           "hbm_bytes_per_launch": rd + wr, "alg_bytes_per_launch": alg,
           "traffic_over_alg": (rd + wr) / alg, "dispatches": [nf, nw]}
    path = os.path.join(ROOT, "profiles", "spmm_mid_n2e6_traffic.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))
    # reorthogonalisation kernels on a REORTH_BLOCKS-block FP32 basis of the
    # same n: the gram reads the basis and W' (FP64), the update reads both
    # and writes W'
    n, b, M = H.n, w.nvec, REORTH_BLOCKS * w.nvec
    kern = {"gram": ("k_gram_mfma8", 4 * n * M + 8 * n * b),
            "update": ("k_update_v<float, double, double", 4 * n * M + 16 * n * b)}
    rr = {"workload": "FP32 basis of %d blocks of %d vectors, n=%d; FP64 W'" % (REORTH_BLOCKS, b, n),
          "tallskinny_source_hash": source_hash("tallskinny.hip"),
          "fetch_scale": fetch_scale, "write_scale": write_scale}
    for name, (match, alg_b) in kern.items():
        f_k, nf_k = _per_dispatch(fr, "FETCH_SIZE", match)
        w_k, nw_k = _per_dispatch(wr_, "WRITE_SIZE", match)
        rd_k, wr_k = f_k * 1024.0 * fetch_scale, w_k * 1024.0 * write_scale
        rr[name] = {"kernel_match": match, "fetch_kib": f_k, "write_kib": w_k,
                    "hbm_read_bytes": rd_k, "hbm_write_bytes": wr_k, "alg_bytes": alg_b,
                    "traffic_over_alg": (rd_k + wr_k) / alg_b, "dispatches": [nf_k, nw_k]}
    path = os.path.join(ROOT, "profiles", "reorth_mid_n2e6_traffic.json")
    with open(path, "w") as f:
        json.dump(rr, f, indent=1)
    print(json.dumps(rr))


def kernels_only(torch, bbl, Hd, b, iters=10):
    V = torch.randn((Hd.n, b), dtype=torch.float32, device="cuda")
    W = torch.empty_like(V)
    plan = bbl.spmm_plan(Hd, b)
    for _ in range(iters):
        bbl.spmm_planned(plan, V, W)
    Xb = torch.randn((REORTH_BLOCKS, Hd.n, b), dtype=torch.float32, device="cuda")
    Y = torch.randn((Hd.n, b), dtype=torch.float64, device="cuda")
    for _ in range(3):
        bbl.gram(Xb, REORTH_BLOCKS, b, Y)
    C = torch.randn((REORTH_BLOCKS * b, b), dtype=torch.float64, device="cuda")
    Y2 = torch.empty_like(Y)
    for _ in range(3):
        bbl.block_update(Xb, REORTH_BLOCKS, b, C, -1.0, Y, 1.0, Y2)
    a = torch.randn(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    c = torch.empty_like(a)
    for _ in range(iters):
        torch.neg(a, out=c)
    torch.cuda.synchronize()
    log("kernels-only done")


def compare_pivots(torch, bbl, weights, m_max, sweep=False, n_trunc=0, feature_vectors=0):
    import synthgen
    w = synthgen.WORKLOADS["apply_n5e6"]
    t0 = time.time()
    H = load_matrix(w)
    log("apply matrix n=%d nnz=%d ready in %.1f s" % (H.n, H.nnz, time.time() - t0))
    Hd = bbl.DeviceCSR.from_host(H, "float32", block_rows=w.R)
    params = torch.from_numpy(np.load(weights, allow_pickle=False)).cuda()
    b, k, R = w.nvec, w.k, w.R
    nt = n_trunc or w.n_trunc  # truncation rows (default: 1 % of n)
    fv = feature_vectors       # truncated vectors behind P_D (0: the default 20)
    arms = {}

    def run(name, make):
        torch.cuda.synchronize()
        t = time.perf_counter()
        P, info = make()
        torch.cuda.synchronize()
        tp = time.perf_counter() - t
        plan = bbl.spmm_plan(Hd, b)
        r = bbl.block_lanczos(Hd, P, k, w.tol, m_max=m_max, seed=w.seed, spmm_plan=plan)
        torch.cuda.synchronize()
        tt = time.perf_counter() - t
        info = dict(info, overlap=pivot_overlap(bbl, r.eigvecs, P))
        arms[name] = dict(info, iters=r.stats["iters"], spmm_calls=r.stats["spmm_calls"],
                          converged=bool(r.converged), pivot_s=tp, tts_s=tt,
                          eigvals=[float(x) for x in r.eigvals],
                          max_resid_over_hnorm=float(np.max(r.residuals) / r.stats["hnorm_est"]))
        log("%s: iters=%d pivot %.2f s total %.2f s converged=%s %s" %
            (name, r.stats["iters"], tp, tt, r.converged, info))

    # full-width products of each pivot's construction, in b-wide SpMM units:
    # the learned block needs H P and H Y at width 20 and two width-b checks
    run("random", lambda: (bbl.random_pivot(H.n, b, synthgen.pivot_key(w.seed)),
                           {"pivot_full_spmm": 0}))

    def boot():
        P, st = bbl.bootstrap_pivot(Hd, nt, b, w.tol, m_max=m_max, seed=w.seed)
        return P, {"pivot_full_spmm": 0, "truncated_iters": st["iters"]}
    run("bootstrap", boot)

    def variant_d():
        f = bbl.pivot_features(Hd, nt, R, w.tol, m_max=m_max, seed=w.seed, feature_vectors=fv)
        return f["p_d"][:, :b].contiguous(), {"pivot_full_spmm": 4,
                                              "truncated_iters": f["stats"]["iters"]}
    run("variant_d", variant_d)

    def learned():
        P, info = bbl.learned_pivot(Hd, params, nt, R, b, k, w.tol, m_max=m_max,
                                    seed=w.seed, feature_vectors=fv)
        return P, {"pivot_full_spmm": 6, "choice": info["choice"],
                   "rr_sums": [float(x) for x in info["rr_sums"]],
                   "truncated_iters": info["stats"]["iters"]}
    run("learned", learned)
    ref = np.array(arms["bootstrap"]["eigvals"])
    for a in arms.values():
        a["max_eig_rel_diff_vs_bootstrap"] = float(np.max(np.abs(np.array(a["eigvals"]) - ref) /
                                                          np.abs(ref)))
    if sweep:
        arms["spmm_block_sweep"] = spmm_block_sweep(torch, bbl, H, R, Hd)
    print(json.dumps({"mode": "compare-pivots", "workload": "sectored symmetric CSR n=5e6, "
                      "~300 nnz/row, FP32, b=k=10, tol=1e-6, truncation %d rows, P_D from %d "
                      "truncated vectors, seed 200" % (nt, fv or 20),
                      "n": H.n, "nnz": H.nnz, "m_max": m_max, "weights": os.path.basename(weights),
                      "arms": arms}), flush=True)


def pivot_overlap(bbl, X, P):
    """Cosines of the principal angles between the converged eigenvectors
    and the pivot block (the library's overlap diagnostic)."""
    cos, _ = bbl.pivot_overlap(X.contiguous(), P.contiguous())
    return [float(x) for x in cos]


def independent_residuals(torch, Hd, X, theta, chunk=400_000_000):
    """||H x_i - theta_i x_i||_2 in float64 through torch's sparse CSR product
    (the vendor sparse library), independent of this library's kernels: the
    matrix is taken in row chunks of at most `chunk` stored entries, its
    float32 values promoted to float64."""
    rp = Hd.row_ptr
    n, k = X.shape
    th = torch.as_tensor(np.asarray(theta, dtype=np.float64), device=X.device)
    acc = torch.zeros(k, dtype=torch.float64, device=X.device)
    rp_h = rp.cpu().numpy()
    r0 = 0
    while r0 < n:
        r1 = int(np.searchsorted(rp_h, rp_h[r0] + chunk, side="right")) - 1
        r1 = min(n, max(r1, r0 + 1))
        p0, p1 = int(rp_h[r0]), int(rp_h[r1])
        crow = (rp[r0:r1 + 1] - p0).to(torch.int32)
        A = torch.sparse_csr_tensor(crow, Hd.col[p0:p1], Hd.val[p0:p1].double(), size=(r1 - r0, n))
        Y = torch.matmul(A, X) - X[r0:r1] * th
        acc += (Y * Y).sum(0)
        del A, Y, crow
        r0 = r1
    return acc.sqrt().cpu().numpy()


def parlett_bounds(theta, resid):
    """Quadratic residual bound on the eigenvalue error of each Ritz value,
    ||r_i||^2 / gap_i (Parlett, The Symmetric Eigenvalue Problem, Thm 11.7.1),
    with gap_i taken from the neighbouring computed Ritz values (an estimate:
    the true gap to the rest of the spectrum is not known without the
    oracle)."""
    th = np.asarray(theta, dtype=np.float64)
    out = []
    for i in range(len(th)):
        others = np.delete(th, i)
        gap = float(np.min(np.abs(others - th[i]))) if len(others) else float("inf")
        out.append(float(resid[i]) ** 2 / gap if gap > 0 else float("inf"))
    return out


def reorth_flops(n, b, iters, basis_blocks, restarts, keep, m_max):
    """FP64 flops of the Gram-Schmidt sweep (gram and update, 2 n M b each for
    M = J b stored columns) over every block iteration the solve ran."""
    q = keep // b if restarts else 0
    Js = list(range(m_max)) if restarts else list(range(basis_blocks))
    for c in range(restarts):
        last = (c == restarts - 1)
        Js += list(range(q, basis_blocks if last else m_max))
    return sum(4.0 * n * (J + 1) * b * b for J in Js[:iters])


def large_workload(torch, bbl, name, args):
    """C3 (n = 2e7, ~400 nnz/row, b = 16, k = 10) or C5 (n = 1e8, ~50 nnz/row,
    50/50 locality, b = k = 8): at most m_max = 40 stored FP32 blocks with
    thick restart, bootstrapped pivot from the leading n_trunc rows.  One
    timed solve (pivot + solve + Ritz vectors + FP64 residual, matrix
    resident); residuals recomputed in FP64 by the vendor sparse library;
    eigenvalue accuracy certified by the quadratic residual bound."""
    import synthgen
    w = synthgen.WORKLOADS[name]
    b, k, keep = w.nvec, w.k, args.restart_keep
    t0 = time.time()
    H = w.generate(values="f32", verbose=True)
    log("%s: n=%d nnz=%d (%.1f nnz/row) generated in %.1f s" % (name, H.n, H.nnz, H.nnz / H.n,
                                                                 time.time() - t0))
    t0 = time.time()
    Hd = bbl.DeviceCSR.from_host(H, "float32", block_rows=w.R)
    torch.cuda.synchronize()
    log("uploaded in %.1f s" % (time.time() - t0))
    ws = torch.empty(bbl.lanczos_workspace_bytes(H.n, b, k, w.m_max, bbl.BBL_F32, keep),
                     dtype=torch.uint8, device="cuda")
    log("workspace %.1f GB" % (ws.numel() / 1e9))
    res = {}
    plan = None
    for rep_i in range(max(1, args.steps)):
        del plan
        torch.cuda.synchronize()
        t = time.perf_counter()
        plan = None if args.plain_spmm else bbl.spmm_plan(Hd, b)
        torch.cuda.synchronize()
        tplan = time.perf_counter() - t
        P, pst = bbl.bootstrap_pivot(Hd, w.n_trunc, b, w.tol, m_max=w.m_max, seed=w.seed,
                                     restart_keep=keep)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t - tplan
        log("plan %.2f s (%s); pivot: %.2f s, truncated iters %d restarts %d converged %d" %
            (tplan, "none" if plan is None else "%d sets of %d blocks, %.1f GB" %
             (plan.c.nsets, plan.slots, plan.mem.numel() / 1e9),
             tp, pst["iters"], pst["restarts"], pst["converged"]))
        r = bbl.block_lanczos(Hd, P, k, w.tol, m_max=w.m_max, seed=w.seed, workspace=ws,
                              restart_keep=keep, time_phases=True, spmm_plan=plan)
        torch.cuda.synchronize()
        tts = time.perf_counter() - t
        st = r.stats
        log("solve %d: tts %.2f s iters %d restarts %d converged %s" %
            (rep_i, tts, st["iters"], st["restarts"], r.converged))
        res = {"tts_s": tts, "pivot_s": tp, "plan_s": tplan, "stats": st, "pivot_stats": pst,
               "r": r}
    r, st = res["r"], res["stats"]
    alg = spmm_bytes(H.n, H.nnz, b, 4, 4)
    t_spmm = st["spmm_ms"] / 1e3 / max(st["spmm_timed"], 1)
    log("FP64 residuals through the vendor sparse library ...")
    t0 = time.time()
    del ws
    torch.cuda.empty_cache()
    hres = independent_residuals(torch, Hd, r.eigvecs, r.eigvals)
    log("residuals in %.1f s" % (time.time() - t0))
    hn = st["hnorm_est"]
    fl = reorth_flops(H.n, b, st["iters"], st["basis_blocks"], st["restarts"], keep, w.m_max)
    out = {
        "mode": "large", "workload": name,
        "config": "sectored symmetric CSR n=%d, %.0f nnz/row, sectors of %d, p=%.1f, FP32 "
                  "values and basis, b=%d, k=%d, tol=%g, <= %d stored blocks, thick restart "
                  "keeping %d Ritz vectors, bootstrap from the leading %d rows" %
                  (H.n, H.nnz / H.n, w.R, w.p, b, k, w.tol, w.m_max, keep, w.n_trunc),
        "n": H.n, "nnz": H.nnz, "tts_s": res["tts_s"], "pivot_s": res["pivot_s"],
        "converged": bool(r.converged), "iters": st["iters"], "restarts": st["restarts"],
        "vector_equiv_iters": st["iters"] * b, "spmm_calls": st["spmm_calls"],
        "pivot_iters": res["pivot_stats"]["iters"],
        "pivot_spmm_calls": res["pivot_stats"]["pivot_spmm_calls"],
        "eigvals": [float(x) for x in r.eigvals],
        "resid_over_hnorm_device": [float(x) / hn for x in r.residuals],
        "resid_over_hnorm_fp64_vendor_sparse": [float(x) / hn for x in hres],
        "parlett_bound_abs": parlett_bounds(r.eigvals, hres),
        "plan_s": res["plan_s"],
        "spmm": {"kernel": "plain CSR (k_spmm)" if plan is None else
                 "multi-set planned (k_spmm_pipe_ms + k_spmm_rest), %d sets of %d blocks"
                 % (plan.c.nsets, plan.slots) if plan.c.nsets else "planned (k_spmm_pipe12 + "
                 "k_spmm_rest)", "alg_bytes_per_call": alg,
                 "ms_per_call": t_spmm * 1e3, "alg_GBps": alg / t_spmm / 1e9,
                 "frac_hbm_peak": alg / t_spmm / HBM_PEAK, "calls_timed": st["spmm_timed"]},
        "phases_ms": {f: st[f] for f in ("spmm_ms", "t_threeterm_ms", "t_reorth_ms", "t_qr_ms",
                                          "t_eig_ms", "t_restart_ms")},
        "reorth_fp64": {"flops": fl, "TFLOPs": fl / (st["t_reorth_ms"] / 1e3) / 1e12,
                        "frac_fp64_peak": fl / (st["t_reorth_ms"] / 1e3) / FP64_PEAK},
        "device_GB": torch.cuda.max_memory_allocated() / 1e9,
    }
    if args.spmm_sweep:
        out["spmm_block_sweep"] = spmm_block_sweep(torch, bbl, H, w.R, Hd)
    print(json.dumps(out), flush=True)


SWEEP_WIDTHS = (1, 2, 4, 8, 12, 16, 32)


def spmm_block_sweep(torch, bbl, H, R, Hb=None):
    """SpMM time per operation (one matrix element times one vector) for
    block widths 1..32, plain CSR kernel and, where a plan exists, the planned
    kernel (the GPU analogue of the paper's block-size tables)."""
    if Hb is None:
        Hb = bbl.DeviceCSR.from_host(H, "float32", block_rows=R)
    Hp = bbl.DeviceCSR(Hb.n, Hb.row_ptr, Hb.col, Hb.val, 0)
    out = {}
    for b in SWEEP_WIDTHS:
        V = torch.randn((H.n, b), dtype=torch.float32, device="cuda")
        W = torch.empty_like(V)
        t_plain = time_kernel(torch, lambda: bbl.spmm(Hp, V, W), 10)
        rec = {"plain_ms": t_plain * 1e3, "plain_ns_per_op": t_plain / (H.nnz * b) * 1e9,
               "plain_alg_GBps": spmm_bytes(H.n, H.nnz, b, 4, 4) / t_plain / 1e9}
        try:
            plan = bbl.spmm_plan(Hb, b)
            t_pl = time_kernel(torch, lambda: bbl.spmm_planned(plan, V, W), 10)
            rec.update({"planned_ms": t_pl * 1e3, "planned_ns_per_op": t_pl / (H.nnz * b) * 1e9,
                        "planned_alg_GBps": spmm_bytes(H.n, H.nnz, b, 4, 4) / t_pl / 1e9,
                        "plan_slots": plan.slots})
            del plan
        except (bbl.BblError, RuntimeError):
            pass
        del V, W
        torch.cuda.empty_cache()
        out[str(b)] = rec
        log("b=%d %s" % (b, json.dumps(rec)))
    return out


def time_kernel(torch, fn, iters):
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    start.record()
    for _ in range(iters):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / 1e3 / iters


def host_info():
    import platform
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = None
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            q, per = f.read().split()[:2]
            quota = None if q == "max" else float(q) / float(per)
    except (OSError, ValueError):
        pass
    return {"cpu_model": model or platform.processor(), "cpus_affinity": aff,
            "cpu_count": os.cpu_count(), "cgroup_cpu_quota": quota,
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS"),
            "OMP_PROC_BIND": os.environ.get("OMP_PROC_BIND")}


def cpu_baseline(H, w, pivot_np, gpu_iters):
    """The FP64 oracle on the host cores, as it stands:
    * the small FP64 workload (n = 2e4, b = k = 4, tol 1e-8, bootstrap from the
      leading 2000 rows) solved in full and timed;
    * the benchmark workload on a bounded sample: the truncated pivot solve
      timed in full; block iterations m = 6 and m = 18 of the solve from the
      same pivot on the same float32-rounded matrix timed, fitted as a + c j
      per block (products, recurrence, reorthogonalisation against j blocks);
      the oracle's dense band eigensolve of each block, O((j b)^3), timed at
      four sizes up to the final 8 x iterations and summed over the GPU's
      iteration count with a cubic fit; plus one explicit-residual product.
    `value` is that estimate of the full solve, in seconds."""
    import oracle
    import synthgen
    info = host_info()
    threads = int(info["OMP_NUM_THREADS"] or info["cpu_count"] or 1)
    w1 = synthgen.WORKLOADS["small_fp64_n2e4"]
    H1 = w1.generate()
    t0 = time.perf_counter()
    P1 = oracle.bootstrap_pivot(H1, w1.n_trunc, w1.nvec)
    r1 = oracle.block_lanczos(H1, P1, w1.k, w1.tol, w1.m_max)
    t_small = time.perf_counter() - t0
    H32 = H.as_float32_values()
    t0 = time.perf_counter()
    oracle.bootstrap_pivot(H32, w.n_trunc, w.nvec, tol=w.tol, m_max=w.m_max, seed=w.seed)
    t_piv = time.perf_counter() - t0
    m1, m2 = 6, 18
    t0 = time.perf_counter()
    oracle.block_lanczos(H32, pivot_np, w.k, 1e-300, m1, seed=w.seed)
    t1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.block_lanczos(H32, pivot_np, w.k, 1e-300, m2, seed=w.seed)
    t2 = time.perf_counter() - t0
    # t(m) = a m + c m^2 / 2  (block j costs a + c j)
    A = np.array([[m1, m1 * m1 / 2.0], [m2, m2 * m2 / 2.0]])
    a, c = np.linalg.solve(A, np.array([t1, t2]))
    a, c = max(a, 0.0), max(c, 0.0)
    m, b = gpu_iters, w.nvec
    rng = np.random.default_rng(0)
    sizes = [int(round(m * b * f)) for f in (0.25, 0.5, 0.75, 1.0)]
    te = []
    for N in sizes:
        S = rng.standard_normal((N, N))
        S = S + S.T
        t0 = time.perf_counter()
        np.linalg.eigh(S)
        te.append(time.perf_counter() - t0)
    # t_eigh(N) = e N^3, least squares over the four sizes
    N3 = np.array(sizes, dtype=np.float64) ** 3
    e = float(np.dot(N3, te) / np.dot(N3, N3))
    t_eig = sum(e * float(j * b) ** 3 for j in range(1, m + 1))
    est = t_piv + a * m + c * m * m / 2.0 + t_eig + a
    return {
        "value": est, "unit": "s", "cores": threads, "kind": "oracle",
        "sample": ("FP64 oracle (C loops + numpy), %s, %s threads: the n=2e4 FP64 workload "
                   "solved in full in %.2f s (%d blocks); for this workload the truncated "
                   "pivot solve timed in full (%.1f s), block iterations m=%d (%.1f s) and "
                   "m=%d (%.1f s) timed and fitted a+c*j per block, dense band eigensolves "
                   "timed at N=%s (%s s) and fitted e*N^3, all summed to the GPU's %d "
                   "iterations" % (info["cpu_model"], threads, t_small, r1.iters, t_piv, m1, t1,
                                   m2, t2, sizes, ["%.2f" % x for x in te], m)),
        "small_fp64_full_s": t_small, "small_fp64_eigvals": [float(x) for x in r1.eigvals],
        "host": info,
        "model_terms_s": {"pivot": t_piv, "blocks_linear": a * m + c * m * m / 2.0 + a,
                          "band_eigensolves": t_eig},
    }


def small_fp64_leg(torch, bbl):
    """The small FP64 workload on the GPU (n = 2e4, ~40 nnz/row, b = k = 4,
    tol 1e-8, bootstrap pivot from the leading 2000 rows, plain CSR SpMM: the
    plan's one workgroup per sector of 400 rows gives 50 workgroups, too few
    to fill the chip, 17.8 against 15.9 ms per solve):
    time to solution of a warm solve (pivot + solve + Ritz vectors + explicit
    residual), iterations, eigenvalues and residuals; the oracle's solve of
    the same matrix (CPU baseline leg) gives its eigenvalue error."""
    import synthgen
    w1 = synthgen.WORKLOADS["small_fp64_n2e4"]
    H1 = w1.generate()
    Hd1 = bbl.DeviceCSR.from_host(H1, "float64", block_rows=w1.R)
    res = None
    for _ in range(2):  # warm, then timed
        torch.cuda.synchronize()
        t = time.perf_counter()
        P1, _st = bbl.bootstrap_pivot(Hd1, w1.n_trunc, w1.nvec, w1.tol, m_max=w1.m_max,
                                      seed=w1.seed)
        r1 = bbl.block_lanczos(Hd1, P1, w1.k, w1.tol, m_max=w1.m_max, seed=w1.seed)
        torch.cuda.synchronize()
        res = (time.perf_counter() - t, r1)
    tts, r1 = res
    return {"tts_s": tts, "iters": r1.stats["iters"], "converged": bool(r1.converged),
            "eigvals": [float(x) for x in r1.eigvals],
            "max_resid_over_hnorm": float(np.max(r1.residuals) / r1.stats["hnorm_est"])}


def fp64_arm(torch, bbl, H, w, P, r32, spmm_iters):
    """The same workload with float64 values, basis and products, through the
    plain CSR kernel and through the planned SpMM (the pipelined passes on
    rows of doubles): time to solution, SpMM algorithmic GB/s against
    nnz*12 + 8(n+1) + 2*n*b*8 bytes per call, and the eigenvalue difference
    from the float32 solve."""
    Hd64 = bbl.DeviceCSR.from_host(H, "float64", block_rows=w.R)
    b, k = w.nvec, w.k
    plan = bbl.spmm_plan(Hd64, b)
    ws = torch.empty(bbl.lanczos_workspace_bytes(H.n, b, k, w.m_max, bbl.BBL_F64),
                     dtype=torch.uint8, device="cuda")
    out = {}
    for name, pl in (("plain", None), ("planned", plan)):
        bbl.block_lanczos(Hd64, P, k, w.tol, m_max=w.m_max, seed=w.seed, workspace=ws,
                          spmm_plan=pl)  # warm
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = bbl.block_lanczos(Hd64, P, k, w.tol, m_max=w.m_max, seed=w.seed, workspace=ws,
                              time_spmm=True, spmm_plan=pl)
        torch.cuda.synchronize()
        tt = time.perf_counter() - t
        alg = spmm_bytes(H.n, H.nnz, b, 8, 8)
        t_sp = r.stats["spmm_ms"] / 1e3 / max(r.stats["spmm_timed"], 1)
        out[name] = {"solve_s": tt, "iters": r.stats["iters"], "converged": bool(r.converged),
                     "spmm_ms_per_call": t_sp * 1e3, "spmm_alg_GBps": alg / t_sp / 1e9,
                     "spmm_frac_hbm_peak": alg / t_sp / HBM_PEAK, "alg_bytes_per_call": alg,
                     "eigvals": [float(x) for x in r.eigvals],
                     "max_eig_rel_diff_fp32_vs_fp64":
                         float(np.max(np.abs(r32.eigvals - r.eigvals) / np.abs(r.eigvals))),
                     "max_resid_over_hnorm": float(np.max(r.residuals) / r.stats["hnorm_est"])}
        log("fp64 arm (%s): %s" % (name, json.dumps(out[name])))
    del ws, plan, Hd64
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--random-arm", action="store_true",
                    help="also solve once from a random pivot and report its counts")
    ap.add_argument("--spmm-iters", type=int, default=20)
    ap.add_argument("--kernels-only", action="store_true",
                    help="run the SpMM, gram and calibration copy only (counter runs)")
    ap.add_argument("--traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the SpMM HBM traffic record from two rocprofv3 --pmc runs")
    ap.add_argument("--compare-pivots", action="store_true",
                    help="random / bootstrap / variant D / learned pivots on the n=5e6 instance")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2210_15763_amd", "weights",
                                                      "pivot_mlp_sectored.npy"))
    ap.add_argument("--compare-m-max", type=int, default=300)
    ap.add_argument("--compare-trunc", type=int, default=0,
                    help="--compare-pivots: truncation rows (default 50,000, 1 %% of n)")
    ap.add_argument("--feature-vectors", type=int, default=0,
                    help="--compare-pivots: truncated vectors behind P_D, 10..32 (default 20)")
    ap.add_argument("--spmm-sweep", action="store_true",
                    help="SpMM time per operation for block widths 1..16 (plain and planned)")
    ap.add_argument("--workload", default=WORKLOAD,
                    help="mid_n2e6 (the timed benchmark) or large_n2e7 / stress_n1e8 (one "
                         "thick-restarted solve, reported on its own JSON line)")
    ap.add_argument("--plain-spmm", action="store_true",
                    help="large workloads: the plain CSR kernel instead of the planned one")
    ap.add_argument("--restart-keep", type=int, default=32,
                    help="Ritz vectors kept by thick restart (large workloads)")
    ap.add_argument("--no-fp64-arm", action="store_true",
                    help="skip the float64 solve of the same workload")
    ap.add_argument("--single-vector-arm", action="store_true",
                    help="also solve with block size 1 (the single-vector method) from a "
                         "random start and report vector-equivalent iterations")
    args = ap.parse_args()
    if args.traffic:
        write_traffic(*args.traffic)
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the hot path has no multi-GPU build; "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import synthgen
    import paper_2210_15763_amd as bbl
    bbl.load_library()
    if args.compare_pivots:
        compare_pivots(torch, bbl, args.weights, args.compare_m_max, args.spmm_sweep,
                       args.compare_trunc, args.feature_vectors)
        return
    if args.workload != WORKLOAD:
        large_workload(torch, bbl, args.workload, args)
        return
    w = synthgen.WORKLOADS[WORKLOAD]
    t0 = time.time()
    H = load_matrix(w)
    log("matrix n=%d nnz=%d (%.1f nnz/row) ready in %.1f s" % (H.n, H.nnz, H.nnz / H.n,
                                                               time.time() - t0))
    # locality hint: aligned sectors of w.R rows hold most of every row's columns
    Hd = bbl.DeviceCSR.from_host(H, "float32", block_rows=w.R)
    torch.cuda.synchronize()
    b, k = w.nvec, w.k
    if args.kernels_only:
        kernels_only(torch, bbl, Hd, b)
        return

    ws_l = torch.empty(bbl.lanczos_workspace_bytes(H.n, b, k, w.m_max, bbl.BBL_F32),
                       dtype=torch.uint8, device="cuda")

    plan_ms = []
    side = torch.cuda.Stream()  # default priority

    def step():
        # the SpMM plan (partner blocks per sector, rows reordered) is rebuilt
        # inside every timed step, so its cost is part of the time to solution;
        # it runs on a second stream beside the bootstrap's truncated solve,
        # which does not need it
        main = torch.cuda.current_stream()
        side.wait_stream(main)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(side):
            e0.record()
            plan = bbl.spmm_plan(Hd, b)
            e1.record()
        plan.mem.record_stream(main)
        P, pst = bbl.bootstrap_pivot(Hd, w.n_trunc, b, w.tol, m_max=w.m_max, seed=w.seed)
        main.wait_stream(side)
        r = bbl.block_lanczos(Hd, P, k, w.tol, m_max=w.m_max, seed=w.seed, workspace=ws_l,
                              time_spmm=True, spmm_plan=plan)
        plan_ms.append(e0.elapsed_time(e1))
        step.plan = plan
        return P, pst, r

    for i in range(args.warmup):
        _, pst, r = step()
        log("warmup %d: iters=%d converged=%s" % (i, r.stats["iters"], r.converged))
    torch.cuda.synchronize()
    times = []
    spmm_ms, spmm_n = 0.0, 0
    for i in range(args.steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        P, pst, r = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        spmm_ms += r.stats["spmm_ms"]
        spmm_n += r.stats["spmm_timed"]
        log("step %d: %.3f s iters=%d pivot_iters=%d converged=%s" %
            (i, times[-1], r.stats["iters"], pst["iters"], r.converged))
    tts = float(np.mean(times))

    # roofline kernel: the SpMM launches of the timed solves (HIP event pairs on
    # the solver's stream), algorithmic bytes per launch / mean launch time
    alg = spmm_bytes(H.n, H.nnz, b, 4, 4)
    t_live = spmm_ms / 1e3 / max(spmm_n, 1)
    achieved = alg / t_live
    traffic = read_traffic(source_hash("spmm.hip"))
    # the same kernel alone, back to back, and the plain CSR kernel, for comparison
    V = torch.randn((H.n, b), dtype=torch.float32, device="cuda")
    W = torch.empty_like(V)
    t_spmm = time_kernel(torch, lambda: bbl.spmm_planned(step.plan, V, W), args.spmm_iters)
    t_plain = time_kernel(torch, lambda: bbl.spmm(Hd, V, W), args.spmm_iters)

    # reorthogonalisation gram on FP64 matrix cores: V_{1:j}^T W' at j = 50
    j = 50
    Xb = torch.randn((j, H.n, b), dtype=torch.float32, device="cuda")
    Y = torch.randn((H.n, b), dtype=torch.float64, device="cuda")
    t_gram = time_kernel(torch, lambda: bbl.gram(Xb, j, b, Y), 5)
    gram_bytes = j * H.n * b * 4 + H.n * b * 8
    gram_flops = 2.0 * H.n * j * b * b

    # the phase split of one more solve with every phase timed (device time;
    # the band eigensolves run beside the recurrence on their own stream)
    P_ph, _ = bbl.bootstrap_pivot(Hd, w.n_trunc, b, w.tol, m_max=w.m_max, seed=w.seed)
    r_ph = bbl.block_lanczos(Hd, P_ph, k, w.tol, m_max=w.m_max, seed=w.seed, workspace=ws_l,
                             time_phases=True, spmm_plan=step.plan)
    phases = {f: r_ph.stats[f] for f in ("spmm_ms", "t_threeterm_ms", "t_reorth_ms", "t_qr_ms",
                                          "t_eig_ms")}
    log("phases: %s" % json.dumps(phases))
    hres = None
    extra = {
        "phases_ms": phases,
        "bootstrap": {"iters": r.stats["iters"], "spmm_calls": r.stats["spmm_calls"],
                      "checks": r.stats["checks"], "deflations": r.stats["deflations"],
                      "reorth_second_passes": r.stats["reorth_second_passes"],
                      "vector_equiv_iters": r.stats["iters"] * b,
                      "pivot_iters": pst["iters"], "pivot_spmm_calls": pst["spmm_calls"],
                      "eigvals": [float(x) for x in r.eigvals],
                      "max_resid_over_hnorm": float(np.max(r.residuals) / r.stats["hnorm_est"]),
                      "converged": bool(r.converged)},
        "spmm": {"in_solve_ms_per_launch": t_live * 1e3, "in_solve_launches": spmm_n,
                 "in_solve_share_of_tts": spmm_ms / 1e3 / max(sum(times), 1e-30),
                 "isolated_ms": t_spmm * 1e3, "isolated_alg_GBps": alg / t_spmm / 1e9,
                 "plain_csr_kernel_ms": t_plain * 1e3, "plan_build_ms": float(np.mean(plan_ms)),
                 "plan_slots": step.plan.slots},
        "reorth_gram_j50": {"ms": t_gram * 1e3, "alg_GBps": gram_bytes / t_gram / 1e9,
                            "fp64_TFLOPs": gram_flops / t_gram / 1e12,
                            "frac_fp64_peak": gram_flops / t_gram / FP64_PEAK},
    }
    # the roofline time to solution: bytes every phase that ran must move at
    # least, over the 8 TB/s peak (the truncated pivot solve included)
    rp = np.asarray(H.row_ptr)
    nt = w.n_trunc
    nnz_t = int(np.count_nonzero(np.asarray(H.col[:rp[nt]]) < nt))
    by_main = solve_bytes(H.n, H.nnz, b, k, r.stats["iters"],
                          r.stats["spmm_calls"] - r.stats["iters"], r.stats["reorth_second_passes"])
    by_piv = solve_bytes(nt, nnz_t, b, b, pst["iters"], pst["spmm_calls"] - pst["iters"], 0)
    extra["roofline_tts"] = {"s": (by_main + by_piv) / HBM_PEAK, "bytes": by_main + by_piv,
                             "main_solve_bytes": by_main, "pivot_solve_bytes": by_piv,
                             "measured_over_roofline": tts / ((by_main + by_piv) / HBM_PEAK)}
    if args.spmm_sweep:
        extra["spmm_block_sweep"] = spmm_block_sweep(torch, bbl, H, w.R, Hd)
    if args.single_vector_arm:
        p1 = bbl.random_pivot(H.n, 1, synthgen.pivot_key(w.seed))
        plan1 = bbl.spmm_plan(Hd, 1)
        torch.cuda.synchronize()
        t = time.perf_counter()
        r1 = bbl.block_lanczos(Hd, p1, k, w.tol, m_max=3000, seed=w.seed, spmm_plan=plan1)
        torch.cuda.synchronize()
        extra["single_vector"] = {"iters": r1.stats["iters"], "vector_equiv_iters": r1.stats["iters"],
                                  "tts_s": time.perf_counter() - t, "converged": bool(r1.converged),
                                  "max_eig_rel_diff_vs_bootstrap":
                                      float(np.max(np.abs(r1.eigvals - r.eigvals) / np.abs(r.eigvals)))}
        log("single-vector: %s" % json.dumps(extra["single_vector"]))
    if args.random_arm:
        Pr = bbl.random_pivot(H.n, b, synthgen.pivot_key(w.seed))
        torch.cuda.synchronize()
        t = time.perf_counter()
        rr = bbl.block_lanczos(Hd, Pr, k, w.tol, m_max=w.m_max, seed=w.seed, spmm_plan=step.plan)
        torch.cuda.synchronize()
        extra["random"] = {"iters": rr.stats["iters"], "spmm_calls": rr.stats["spmm_calls"],
                           "tts_s": time.perf_counter() - t, "converged": bool(rr.converged),
                           "max_eig_rel_diff_vs_bootstrap":
                               float(np.max(np.abs(rr.eigvals - r.eigvals) / np.abs(r.eigvals)))}
    if not args.no_fp64_arm:
        extra["fp64_arm"] = fp64_arm(torch, bbl, H, w, P, r, args.spmm_iters)
    extra["small_fp64"] = small_fp64_leg(torch, bbl)
    log("small FP64 workload: %s" % json.dumps(extra["small_fp64"]))
    # eigenvalue accuracy of this run: FP64 residuals of the returned pairs
    # recomputed by the vendor sparse library, and the quadratic residual
    # bound on each eigenvalue's error
    hres = independent_residuals(torch, Hd, r.eigvecs, r.eigvals)
    extra["accuracy"] = {
        "resid_over_hnorm_fp64_vendor_sparse": [float(x) / r.stats["hnorm_est"] for x in hres],
        "parlett_bound_abs": parlett_bounds(r.eigvals, hres),
        "note": "eigenvalue error vs the exact eigenvalues of the stored FP32 matrix is at most "
                "||r||^2/gap (gap estimated from the neighbouring Ritz values); the FP64 arm "
                "gives the difference from a float64 solve"}
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample) ...")
        cpu = cpu_baseline(H, w, P.cpu().numpy(), r.stats["iters"])
        ref = np.array(cpu["small_fp64_eigvals"])
        got = np.array(extra["small_fp64"]["eigvals"])
        extra["small_fp64"]["max_eig_rel_err_vs_oracle"] = float(np.max(np.abs(got - ref) /
                                                                        np.abs(ref)))

    out = {
        "metric": "time-to-solution, 10 eigpairs @1e-6 resid",
        "value": tts,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": tts * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sectored symmetric CSR n=2e6, ~200 nnz/row, FP32 values, "
                               "b=8, k=10, tol=1e-6, bootstrap pivot from leading 20000 rows",
                   "block_rows_hint": w.R,
                   "n": H.n, "nnz": H.nnz, "nvec": b, "k": k, "tol": w.tol,
                   "n_trunc": w.n_trunc, "m_max": w.m_max, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK,
                     "traffic": traffic, "kernel": "k_spmm_pipe12<8, false, float> + k_spmm_rest<8, false, float>",
                     "alg_bytes_per_launch": alg, "launch_ms": t_live * 1e3},
        "cpu_baseline": cpu,
        "details": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
