"""Benchmark: Frobenius matrices per second for a batch of random smooth plane
quintic curves over F_31 (256 curves per step), plus modular mat-vecs/s.

One step = one cr_frobenius_batch call over the whole batch: host setup,
device reduction of every start term to pole n, device Griffiths-Dwork
assembly, host unscaling and integer L-polynomials.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--no-cpu-baseline] [--no-legs]

Prints one JSON line.  `roofline` describes the reduction kernel (the
dominant one), timed with HIP events on the stream it runs on; `cpu_baseline`
times the CPU oracle on a bounded sample of the same workload; `plain` is the
per-hypersurface path on the same GPU (one cr_frobenius call per item, 64-bit
VALU kernel, depth-first policy) and `learned` the batch under the learned
policy (network trained on the GPU from plain-policy traces of other items).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

INT8_PEAK_TOPS = 5000.0  # MI355X dense int8 MFMA, TOP/s
KERNEL_NAMES = {0: "k_reduce_mfma5", 1: "k_reduce_chains", 2: "k_reduce_mfma", 3: "k_reduce_mfma4",
                4: "k_reduce_quad", 5: "k_reduce_wide"}  # engine that ran


def measured_traffic(kernel, workload):
    """HBM bytes per launch of the reduction kernel from the committed rocprofv3
    counters, if they were taken on the kernel source as it is now."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "%s_%s.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    prof = json.load(open(path))
    src = open(os.path.join(ROOT, prof["kernel_source"]), "rb").read()
    if hashlib.sha256(src).hexdigest() != prof["kernel_source_sha256"]:
        return None
    return prof["traffic_bytes_per_launch"]


def limbs_for(q):
    """Balanced base-256 digits needed for residues mod q."""
    L = 1
    while 256 ** L <= q:
        L += 1
    return L


def _oracle_one(args):
    nv, d, p, c, s_mask, r, n_series = args
    from oracle.frobenius import frobenius
    # under a precision override Q(T) is out of reach: the Frobenius matrix only
    frobenius(nv, d, p, c, S=[i for i in range(nv) if (s_mask >> i) & 1] if s_mask else None,
              r=r or None, N=n_series or None, lpoly=not r)
    return 1


def wfamily(C, w, **kw):
    """The library family of workload w (its S and precision overrides)."""
    return C.family(w.nvars, w.degree, w.s_mask, r=w.r, n_series=w.n_series, **kw)


def run_batch(C, w, fam, primes, coeffs, stream):
    """One cr_frobenius_batch call; every item must succeed, except that under
    a precision override Q(T) may be out of reach (CR_EPRECISION: the
    Frobenius matrix is still computed)."""
    res = C.cr_frobenius_batch(fam, primes, coeffs, stream=stream, want_scaled=False, lpoly_ints=False,
                               raise_on_error=False)
    allowed = (C.CR_OK, C.CR_EPRECISION) if w.r else (C.CR_OK,)
    bad = [(i, int(x)) for i, x in enumerate(res["item_status"]) if int(x) not in allowed]
    if bad or (res["status"] not in allowed):
        raise C.CrError(res["status"], "items failed: %s" % bad[:8])
    return res


def host_info():
    """nproc, CPU model and clock of the host (from /proc/cpuinfo)."""
    info = {"nproc": os.cpu_count()}
    try:
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k = k.strip()
            if k == "model name" and "cpu_model" not in info:
                info["cpu_model"] = v.strip()
            elif k == "cpu MHz" and "cpu_mhz" not in info:
                info["cpu_mhz"] = float(v)
    except OSError:
        pass
    return info


def cpu_baseline(name, items, budget_s=20.0):
    """The CPU oracle timed on the first items of the workload, on a pool of
    host processes (one hypersurface per task, as many processes as the host
    gives this job, at most 16) until ~budget_s of CPU work per process; at
    least one item per process."""
    import multiprocessing as mp
    from paper_2602_24155_amd import workload
    w = workload.WORKLOADS[name]
    cores = max(1, min(16, os.cpu_count() or 1))
    # calibrate on one item, in a child process with a time limit (the oracle
    # needs about ten minutes per cubic threefold)
    ctx = mp.get_context("fork")
    t = time.perf_counter()
    pool = ctx.Pool(1)
    try:
        pool.apply_async(_oracle_one, ((w.nvars, w.degree, items[0][0], items[0][1], w.s_mask, w.r,
                                             w.n_series),)).get(timeout=3 * budget_s)
    except mp.TimeoutError:
        pool.terminate()
        out = {"value": None, "unit": "frobenius_matrices/s", "cores": 1, "kind": "oracle",
               "sample": "none: the oracle did not finish one hypersurface of %s in %.0f s" % (name, 3 * budget_s)}
        out.update(host_info())
        return out
    finally:
        pool.close()
        pool.join()
    per = time.perf_counter() - t
    n = max(cores, min(len(items), int(cores * budget_s / max(per, 1e-3))))
    n = min(n, len(items))
    sample = [(w.nvars, w.degree, p, c, w.s_mask, w.r, w.n_series) for p, c in items[:n]]
    t = time.perf_counter()
    with ctx.Pool(min(cores, n)) as pool:
        done = sum(pool.map(_oracle_one, sample, chunksize=1))
    wall = time.perf_counter() - t
    out = {"value": done / wall, "unit": "frobenius_matrices/s", "cores": min(cores, n), "kind": "oracle",
           "sample": "first %d of the %d %s hypersurfaces, one per task on %d processes "
                     "(exact-integer Python + plain-C oracle, %.1f s wall)" % (n, len(items), name, min(cores, n),
                                                                                wall)}
    out.update(host_info())
    return out


def plain_leg(C, w, items, sample, stream):
    """The per-hypersurface path on the GPU: one cr_frobenius call per item
    (64-bit VALU kernel, depth-first policy), over the first `sample` items."""
    import torch
    fam = wfamily(C, w, policy=C.CR_POLICY_DEPTH_FIRST, engine=C.ENGINE_VALU)
    sub = items[:sample]
    allowed = (C.CR_OK, C.CR_EPRECISION) if w.r else (C.CR_OK,)

    def one(p, c):
        res = C.cr_frobenius(fam, p, c, stream=stream, want_scaled=False, raise_on_error=False)
        if res["status"] not in allowed:
            raise C.CrError(res["status"], C.lib().cr_last_error().decode())
        return res

    try:
        one(sub[0][0], sub[0][1])  # warm up
    except C.CrError as e:  # families the 64-bit kernel does not take (cubic threefolds)
        return {"value": None, "unit": "frobenius_matrices/s", "note": str(e)}
    torch.cuda.synchronize()
    t = time.perf_counter()
    steps = 0
    for p, c in sub:
        steps += one(p, c)["stats"].column_steps
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    return {"value": len(sub) / wall, "unit": "frobenius_matrices/s", "ms_per_matrix": wall / len(sub) * 1e3,
            "matvecs_per_s": steps / wall, "sample": "first %d items, one cr_frobenius call each" % len(sub),
            "engine": "k_reduce_chains (64-bit VALU)", "policy": "depth-first"}


# workloads whose network is trained on the traces of other families: the
# quintic surfaces use a network trained on plane quartics, plane quintics and
# quartic K3 surfaces only
TRAIN_FROM = {"quintic_surfaces_r8": ("quartic_curve_f7", "quintic_curves_mixed", "quartic_k3_mixed")}


def learned_leg(C, w, fam0, items, primes, coeffs, stream, steps, train_from=None):
    """The learned policy on the same batch: the network is trained on the GPU
    (cr_mlp_train) from the plain p-chunk traces of 8 other items (of the
    workload, or of the families TRAIN_FROM names), then the batch is reduced
    under CR_POLICY_LEARNED (judged by the game cost against depth-first and
    p-chunk; the bits are unchanged)."""
    import numpy as np
    import torch
    from paper_2602_24155_amd import workload
    sources = [workload.WORKLOADS[n] for n in (train_from or TRAIN_FROM.get(w.name, (w.name,)))]
    xs, ts = [], []
    for k, ws in enumerate(sources):
        famc = wfamily(C, ws)
        n = 8 // len(sources) + (1 if k < 8 % len(sources) else 0)
        for j in range(ws.count, ws.count + n):
            p, c = workload.first_accepted(ws, j, lambda p_, c_: C.cr_check_smooth(famc, p_, c_))
            x, t = C.cr_trace_policy(famc, p, c)
            xs.append(x)
            ts.append(t)
    x, t = np.concatenate(xs), np.concatenate(ts)
    m = C.Mlp(seed=2)
    t0 = time.perf_counter()
    losses = m.train(x, t, epochs=8, batch=512, lr=2e-3, seed=4, stream=stream)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    fam = wfamily(C, w, policy=C.CR_POLICY_LEARNED, mlp=m, launch=fam0.launch)
    run_batch(C, w, fam, primes, coeffs, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = run_batch(C, w, fam, primes, coeffs, stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    st = res["stats"]
    famp = wfamily(C, w, policy=C.CR_POLICY_P_CHUNK, launch=fam0.launch)
    resp = run_batch(C, w, famp, primes, coeffs, stream)
    m.close()
    return {"value": len(primes) / wall, "unit": "frobenius_matrices/s", "ms_per_step": wall * 1e3,
            "trained_on": [ws.name for ws in sources], "column_steps": st.column_steps,
            "merged_terms": st.merged_terms, "fallbacks": st.fallbacks,
            "p_chunk_column_steps": resp["stats"].column_steps, "p_chunk_merged_terms": resp["stats"].merged_terms,
            "reduce_ms": st.reduce_ms, "p_chunk_reduce_ms": resp["stats"].reduce_ms,
            "train_rows": int(x.shape[0]), "train_s": train_s, "train_loss": [float(losses[0]), float(losses[-1])]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="quintic_curves_p31")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true", help="skip the plain per-hypersurface and learned-policy legs")
    ap.add_argument("--plain-sample", type=int, default=32)
    ap.add_argument("--policy", default="auto", choices=["auto", "depth-first", "p-chunk", "var-by-var"],
                    help="reduction policy; auto = the autotuner's choice (measured before the warmup)")
    ap.add_argument("--launch", default="auto", choices=["auto", "grid", "persistent", "graph"])
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes 5 times (profiler calibration "
                         "of the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        x = torch.empty(args.calibrate_copy // 4, dtype=torch.int32, device="cuda").fill_(1)
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": args.calibrate_copy}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the hypersurfaces of a batch are independent; see DESIGN.md for how it would shard)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2602_24155_amd import crfrob as C
    from paper_2602_24155_amd import workload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    w = workload.WORKLOADS[args.workload]
    fam = wfamily(C, w)
    items = [workload.first_accepted(w, j, lambda p, c: C.cr_check_smooth(fam, p, c)) for j in range(w.count)]
    primes = np.asarray([p for p, _ in items], dtype=np.int32)
    coeffs = np.asarray([c for _, c in items], dtype=np.uint32)
    pol_names = ["depth-first", "p-chunk", "var-by-var", "learned"]
    launch_names = ["grid", "persistent", "graph"]
    tuning = None
    if args.policy == "auto" or args.launch == "auto":
        tu = C.cr_autotune(fam, primes, coeffs, trials=2, stream=stream)
        tuning = {"%s/%s" % (pol_names[k // 3], launch_names[k % 3]): round(tu.ms[k], 2)
                  for k in range(12) if tu.ms[k] > 0}
        shape_names = ["auto/1", "auto/2", "single-tile/1", "single-tile/2", "lds-gather/1", "quad/1", "quad/2",
                       "valu/1"]
        tuning.update({"shape %s" % shape_names[k]: round(tu.shape_ms[k], 2) for k in range(8) if tu.shape_ms[k] > 0})
        if args.policy == "auto":
            fam.policy = tu.best_policy
        if args.launch == "auto":
            fam.launch = tu.best_launch
        if args.policy == "auto" and args.launch == "auto":
            fam.engine = tu.best_engine
            fam.grid = tu.best_grid
    if args.policy != "auto":
        fam.policy = pol_names.index(args.policy)
    if args.launch != "auto":
        fam.launch = launch_names.index(args.launch)

    for _ in range(args.warmup):
        run_batch(C, w, fam, primes, coeffs, stream)
    torch.cuda.synchronize()
    tot = {"reduce_ms": 0.0, "combine_ms": 0.0, "psi_ms": 0.0, "assemble_ms": 0.0, "setup_ms": 0.0, "finish_ms": 0.0}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = run_batch(C, w, fam, primes, coeffs, stream)
        for k in tot:
            tot[k] += getattr(res["stats"], k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = res["stats"]
    wall = t1 - t0
    value = len(items) * args.steps / wall
    _nco, s, b = C.cr_query_dims(w.nvars, w.degree)
    # algorithmic work of one step: column_steps products s x s . s mod p^M,
    # priced as int8 MFMA ops with L balanced base-256 digits per residue,
    # item by item (the host plan gives each item's column steps)
    work_p = {}
    for p in sorted(set(int(q) for q in primes)):
        _r, _N, M = C.cr_precision(fam, p)
        L = limbs_for(p ** M)
        work_p[p] = 2 * s * s * L * L
    work = None
    if fam.policy != C.CR_POLICY_LEARNED:
        cs = [C.cr_policy_cost(fam, int(p), c).column_steps for p, c in items]
        if sum(cs) == st.column_steps:
            work = sum(k * work_p[int(p)] for k, (p, _c) in zip(cs, items))
    if work is None:  # the average over the batch's primes
        work = st.column_steps * sum(work_p[int(q)] for q in primes) / len(primes)
    work_per_colstep = work / st.column_steps
    red_s = tot["reduce_ms"] / 1e3 / args.steps
    achieved = work / red_s / 1e12
    kname = KERNEL_NAMES.get(st.engine, "?") + ("_persistent" if st.engine == 3 and fam.launch > 0 else "")
    line = {
        "metric": "Frobenius matrices/sec (batched quintic curves, p=31) + modular matvecs/sec vs plain",
        "value": value,
        "unit": "frobenius_matrices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64 residues mod p^M (int8-limb / int32 exact products)",
        "data": "synthetic: seeded random dense smooth hypersurfaces of the workload, coefficients uniform in F_p",
        "config": {"workload": args.workload, "count": len(items), "nvars": w.nvars, "degree": w.degree,
                   "primes": sorted(set(int(q) for q in primes)), "policy": pol_names[fam.policy],
                   "launch": launch_names[fam.launch], "engine": fam.engine, "grid": fam.grid,
                   "autotune_ms_per_call": tuning,
                   "start_blocks": st.start_blocks, "column_steps_per_step": st.column_steps,
                   "vectors_per_step": st.vectors, "merged_terms_per_step": st.merged_terms},
        "matvecs_per_s": st.column_steps / red_s,
        "breakdown_ms": {k: v / args.steps for k, v in tot.items()},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": INT8_PEAK_TOPS, "unit": "TOP/s",
                     "frac": achieved / INT8_PEAK_TOPS,
                     "traffic": measured_traffic(kname, args.workload),
                     "kernel": kname, "launches_per_step": st.reduce_launches,
                     "avg_launch_ms": tot["reduce_ms"] / args.steps / max(1, st.reduce_launches),
                     "work_per_column_step_int8_ops": work_per_colstep},
    }
    if w.r:  # precision override: the Frobenius matrices mod p^M, Q(T) out of reach
        line["config"]["precision"] = {"r": w.r, "n_series": w.n_series,
                                       "M": {int(p): C.cr_precision(fam, int(p))[2] for p in set(primes.tolist())}}
    if not args.no_legs:
        line["plain"] = plain_leg(C, w, items, args.plain_sample, stream)
        line["learned"] = learned_leg(C, w, fam, items, primes, coeffs, stream, max(1, args.steps // 2))
        if w.name in TRAIN_FROM:  # the same, with a network trained on other items of this family
            line["learned_same_family"] = learned_leg(C, w, fam, items, primes, coeffs, stream,
                                                      max(1, args.steps // 2), train_from=(w.name,))
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload, items)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
