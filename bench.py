#!/usr/bin/env python3
"""dpXOR benchmark on one MI355X.

Workload (default): a database of N = 2^28 records x 32 B (8 GiB) of seeded
uniform bytes, resident in HBM; Q = 64 Bernoulli(0.5) selection vectors,
resident in HBM, answered in one fused database pass per step (stage-1 scan
+ stage-2 reduction).  The same database is also scanned with a single query
to report the single-query DB GB/s and the batched / single ratio.

Prints one JSON line (rank 0).  `value` is queries/s of the batched step.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0                      # MI355X HBM3E, vendor figure
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12   # 32-bit lane ops/s: 256 CUs x 64 lanes x 2.4 GHz
MFMA_PEAK_TFLOPS = {"int8": 5000.0, "fp4": 10100.0}  # dense, vendor figures

CONFIGS = {
    # name: (n_records, record_bytes, q) -- n<log2 N>r<R>q<Q>
    "n28r32q64": (1 << 28, 32, 64),
    "n28r32q16": (1 << 28, 32, 16),
    "n28r32q512": (1 << 28, 32, 512),
    "n25r32q1": (1 << 25, 32, 1),
    "n23r256q8": (1 << 23, 256, 8),
    "n23r256q64": (1 << 23, 256, 64),
    "n23r256q256": (1 << 23, 256, 256),
}

# The arithmetic is exact GF(2) in every variant: bitwise XOR on 32-bit words,
# or 0/1 operands on the matrix cores with exact integer counts (fp32 counts
# stay below 2^24 per record group) whose parity is the answer bit.
VARIANT_DTYPE = {1: "u32 (bitwise select-XOR, exact GF(2))",
                 2: "gf2-exact (int8 0/1 operands, int32 counts)",
                 3: "gf2-exact (fp4 0/1 operands, fp32 counts <= 2^24)"}


def affinity_threads():
    """Host threads this process may run on."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except (AttributeError, OSError):
        return max(1, os.cpu_count() or 1)


def host_info():
    """The host the CPU baseline runs on: logical CPUs, this process's share, model name."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity_threads": affinity_threads(), "cpu_model": model}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


SCAN_SOURCES = ("pir_kernels.hip", "pir_scan_common.h")


def kernel_source_hash(srcs=SCAN_SOURCES):
    """First 16 hex digits of the SHA-256 of the named kernel sources, concatenated."""
    if isinstance(srcs, str):
        srcs = (srcs,)
    h = hashlib.sha256()
    for src in srcs:
        with open(os.path.join(ROOT, "paper_2509_06514_amd", "csrc", src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def kernel_name(cfg, r, q=64):
    """Name of the stage-1 kernel instance a plan launches for q queries (as profilers
    print it). The split-K kernels' second template argument is the database loads'
    cache policy: 2 (nontemporal) for one 64-query tile, 0 for several."""
    if cfg.variant == 1:
        return f"k_stage1_valu<{cfg.q_tile}, {cfg.unroll}, {'true' if r < 32 else 'false'}>"
    mt = cfg.q_tile // 16
    f4 = "true" if cfg.variant == 3 else "false"
    if cfg.unroll in (2, 3, 4):  # LDS ring of that many stages
        return f"k_stage1_mfma_lds<{mt}, {f4}, {cfg.unroll}>"
    dbp = 0 if (q + cfg.q_tile - 1) // cfg.q_tile > 1 else 2
    if cfg.unroll == 12:  # split K on a 2-stage ring
        return f"k_stage1_mfma_ks<2, {dbp}>"
    if cfg.unroll == 15:  # split K, 2-stage ring, selection words 4 K-steps at a time
        return f"k_stage1_mfma_ksw<{dbp}>"
    if cfg.unroll == 16:  # the same with wave-private database stages
        return f"k_stage1_mfma_ksp<{dbp}>"
    if cfg.unroll == 17:  # the same with the database words loaded into registers
        return f"k_stage1_mfma_ksv<{dbp}>"
    return None


def load_traffic(n, r, q, cfg):
    """HBM bytes per launch from committed rocprofv3 counter runs on this database (2^k records
    of r bytes), if they are for this kernel (same source hash, same kernel instance); else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_dpxor_n{n.bit_length() - 1}r{r}.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    entry = t.get(f"q{q}")
    if not entry or t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    if entry.get("kernel") != kernel_name(cfg, r, q):
        return None
    return entry.get("hbm_bytes_per_launch")


def sample_engine_clock(period_s, stop, out):
    """Append the current engine clock (MHz, the starred level of sysfs
    pp_dpm_sclk) to `out` every period_s seconds until `stop` is set.  It
    reads the first DRM card that has the file, which is the GPU in use only
    where the machine has one GPU (as in the serving sweep's records)."""
    import glob
    paths = glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk")
    if not paths:
        log("serve: no pp_dpm_sclk; engine clock not sampled")
        return
    while not stop.is_set():
        try:
            with open(paths[0]) as f:
                for line in f:
                    if line.rstrip().endswith("*"):
                        out.append(int(line.split(":")[1].strip().lower().split("mhz")[0]))
        except (OSError, ValueError):
            pass
        stop.wait(period_s)


def percentile(xs, f):
    s = sorted(xs)
    k = min(len(s) - 1, max(0, int(round(f * (len(s) - 1)))))
    return s[k]


def time_steps(fn, steps, torch):
    """Run fn() `steps` times between device syncs; per-step device times from events."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [a.elapsed_time(b) for a, b in evs]
    return wall, per


def roofline_for(variant, n, r, q, stage1_ms_avg, traffic, roof=None):
    """Roofline record for the stage-1 kernel of one launch (roof: the measured
    streaming-read roof, reported beside the fraction of the 8 TB/s spec)."""
    alg_bytes = n * r + q * ((n + 7) // 8) + q * r
    t_s = stage1_ms_avg / 1e3
    hbm_time = alg_bytes / (HBM_PEAK_GBS * 1e9)
    if variant == 1:
        ops = q * n * r / 4.0  # one select-XOR per (query, 32-bit database word)
        alu_time = ops / (VALU_PEAK_TOPS * 1e12)
        if alu_time > hbm_time:
            ach = ops / t_s / 1e12
            return {"bound": "alu", "achieved": ach, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                    "frac": ach / VALU_PEAK_TOPS, "traffic": traffic,
                    "algorithmic_ops_per_launch": ops, "avg_launch_ms": stage1_ms_avg}
    else:
        flops = 2.0 * q * n * 8 * r
        dt = "int8" if variant == 2 else "fp4"
        mf_time = flops / (MFMA_PEAK_TFLOPS[dt] * 1e12)
        if mf_time > hbm_time:
            ach = flops / t_s / 1e12
            return {"bound": "mfma", "achieved": ach, "peak": MFMA_PEAK_TFLOPS[dt], "unit": "TFLOP/s",
                    "frac": ach / MFMA_PEAK_TFLOPS[dt], "traffic": traffic,
                    "algorithmic_flops_per_launch": flops, "avg_launch_ms": stage1_ms_avg}
    ach = alg_bytes / t_s / 1e9
    rec = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
           "algorithmic_bytes_per_launch": alg_bytes, "avg_launch_ms": stage1_ms_avg}
    if roof:
        rec["read_roof_gbs"] = roof
        rec["frac_of_read_roof"] = ach / roof
    return rec


def cpu_baseline(db_host, sel_rows, n, r, sample_queries, threads):
    """The oracle on the host: `sample_queries` full queries on one thread, then one
    query per thread on `threads` threads at once (the CPU-PIR arrangement of one
    query per core).  The C oracle releases the interpreter lock while it runs.
    Returns the record and the oracle's answers to rows 0 .. threads-1 (row i mod Q)."""
    import threading

    import numpy as np

    import oracle

    t0 = time.perf_counter()
    for i in range(sample_queries):
        oracle.dpxor(db_host, sel_rows[i % len(sel_rows)])
    dt1 = time.perf_counter() - t0
    answers = np.empty((threads, r), np.uint8)

    def one(i):
        answers[i] = oracle.dpxor(db_host, sel_rows[i % len(sel_rows)])

    ths = [threading.Thread(target=one, args=(i,)) for i in range(threads)]
    t0 = time.perf_counter()
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    dtn = time.perf_counter() - t0
    rec = {"value": threads / dtn, "unit": "queries/s", "cores": threads, "kind": "oracle",
           "host": host_info(),
           "build": "gcc -O2 -std=c11 (plain loops, no intrinsics)",
           "sample": f"{threads} full queries (N={n}, R={r}), one per host thread at once, {dtn:.1f} s; "
                     f"single thread: {sample_queries} queries in {dt1:.1f} s",
           "single_thread": {"value": sample_queries / dt1, "unit": "queries/s", "cores": 1,
                             "db_gbs_scanned": sample_queries * n * r / dt1 / 1e9}}
    return rec, answers


def read_roof(ctx, nbytes, torch, reps=5):
    """Practical HBM read roof: the library's streaming-read probe over a fresh
    device buffer of `nbytes`, best mean over unroll x workgroup counts."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0").fill_(0x5A)
    sink = torch.empty((1 << 16, 4), dtype=torch.int32, device="cuda:0")
    best = None
    for unroll in (4, 8, 16):
        for wgs in (1024, 2048, 4096, 8192, 16384, 32768):
            ctx.read_probe_async(src, sink, unroll=unroll, workgroups=wgs)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                ctx.read_probe_async(src, sink, unroll=unroll, workgroups=wgs)
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            gbs = nbytes / (ms / 1e3) / 1e9
            if best is None or gbs > best["achieved_gbs"]:
                best = {"achieved_gbs": gbs, "ms": ms, "unroll": unroll, "workgroups": wgs}
    del src, sink
    best.update({"bytes": nbytes, "frac_of_spec": best["achieved_gbs"] / HBM_PEAK_GBS,
                 "kernel": "k_read_probe (pir_read_probe_async): 16-byte non-temporal loads, "
                           "contiguous range per workgroup"})
    log(f"read roof: {best['achieved_gbs']:.0f} GB/s (unroll {best['unroll']}, {best['workgroups']} workgroups)")
    return best


def phase_breakdown(ctx, db, sel_host, stride, r, qs, steps, torch):
    """Table 1's phases on the device stream for each Q: selection upload from
    pinned host memory, stage 1, stage 2, answer download to pinned host memory
    (HIP events around each phase, means over `steps` rounds)."""
    dev = torch.device("cuda:0")
    out = {}
    for qq in qs:
        h_sel = torch.from_numpy(sel_host[:qq]).pin_memory()
        h_out = torch.empty((qq, r), dtype=torch.uint8).pin_memory()
        d_sel = torch.empty((qq, stride), dtype=torch.uint8, device=dev)
        d_out = torch.empty((qq, r), dtype=torch.uint8, device=dev)
        d_sel.copy_(h_sel)
        db.dpxor_batch_async(d_sel, qq, d_out, sel_stride=stride)
        torch.cuda.synchronize()
        ctx.timing(True)
        ctx.timing_read(reset=True)
        evs = []
        for _ in range(steps):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            e[0].record()
            d_sel.copy_(h_sel, non_blocking=True)
            e[1].record()
            db.dpxor_batch_async(d_sel, qq, d_out, sel_stride=stride)
            e[2].record()
            h_out.copy_(d_out, non_blocking=True)
            e[3].record()
            evs.append(e)
        torch.cuda.synchronize()
        t = ctx.timing_read(reset=True)
        ctx.timing(False)
        h2d = sum(e[0].elapsed_time(e[1]) for e in evs) / steps
        scan = sum(e[1].elapsed_time(e[2]) for e in evs) / steps
        d2h = sum(e[2].elapsed_time(e[3]) for e in evs) / steps
        s1 = t["stage1_ms"] / max(1, t["stage1_launches"])
        s2 = t["stage2_ms"] / max(1, t["stage2_launches"])
        total = h2d + scan + d2h
        rec = {"sel_h2d_ms": h2d, "stage1_ms": s1, "stage2_ms": s2, "answer_d2h_ms": d2h,
               "scan_enqueue_to_done_ms": scan, "total_ms": total,
               "share_pct": {"sel_h2d": 100 * h2d / total, "stage1": 100 * s1 / total,
                             "stage2": 100 * s2 / total, "answer_d2h": 100 * d2h / total},
               "sel_h2d_gbs": qq * stride / (h2d / 1e3) / 1e9}
        out[f"q{qq}"] = rec
        log(f"phases Q={qq}: H2D {h2d:.3f} ms, stage1 {s1:.3f} ms, stage2 {s2:.4f} ms, D2H {d2h:.4f} ms")
        del h_sel, h_out, d_sel, d_out
    return out


# VALU operations per tree-node expansion of the DPF evaluation (AES-128 with
# the T-tables Te0 and Te2: one v_perm per lookup address; per MixColumns
# column one rotation and three XOR instructions; 11 ops per key-schedule round):
#   full (both 128-bit children): 110 key schedule + 1 + 40 round 1 (the second
#     block differs only in column 0) + 512 rounds 2-9 + 56 last round + 18
#     correction words = 737
#   leaf (bit 0 of both children, at the last level): 99 + 3 key schedule + 1 +
#     40 + 448 rounds 2-8 + 16 round 9 (column 0) + 6 last round (byte 0) + 10 = 623
DPF_OPS_FULL = 737
DPF_OPS_LEAF = 623


VARIANT_NAME = {1: "valu_select_xor", 2: "mfma_int8", 3: "mfma_fp4"}


def variant_sweep(ctx, db, d_sel, stride, n, r, q, d_out, torch, pir, reps=3):
    """Best stage-1 time of each kernel family (vector-ALU select-XOR, int8 and fp4 matrix
    cores) for this Q over a fixed candidate list (default record groups), and whether every
    candidate returned the same bytes."""
    import numpy as np
    p2 = 1 << max(0, (q - 1).bit_length())
    fams = {1: [], 2: [], 3: []}
    for qt in (1, 2, 4, 8, 16, 32):
        if min(p2, 8) <= qt <= p2:
            fams[1] += [(qt, u) for u in (2, 4, 8)]
    if q >= 8:
        for v in (2, 3):
            for qt in (16, 32, 64):
                if qt <= max(p2, 16):
                    fams[v] += [(qt, u) for u in (2, 3, 4) + ((15, 16, 17) if v == 3 and qt == 64 else ())]
    ref, same, out = None, True, {}
    for v, cands in fams.items():
        best = None
        for qt, u in cands:
            cfg = pir.KernelCfg(v, qt, u, 0)
            try:
                d_out.fill_(0xEE)
                db.dpxor_batch_async(d_sel, q, d_out, sel_stride=stride, cfg=cfg)
                torch.cuda.synchronize()
            except pir.PirError:
                continue
            got = d_out.cpu().numpy()
            if ref is None:
                ref = got.copy()
            elif not np.array_equal(got, ref):
                same = False
            ctx.timing(True)
            ctx.timing_read(reset=True)
            for _ in range(reps):
                db.dpxor_batch_async(d_sel, q, d_out, sel_stride=stride, cfg=cfg)
            torch.cuda.synchronize()
            t = ctx.timing_read(reset=True)
            ctx.timing(False)
            ms = t["stage1_ms"] / max(1, t["stage1_launches"])
            if best is None or ms < best[0]:
                best = (ms, cfg)
        if best is not None:
            out[VARIANT_NAME[v]] = {"cfg": best[1].as_dict(), "stage1_ms": best[0], "candidates": len(cands),
                                    "roofline": roofline_for(v, n, r, q, best[0], None)}
            log(f"variants Q={q}: {VARIANT_NAME[v]} best {best[0]:.3f} ms {best[1]}")
    return {"families": out, "identical_answers": same, "reps": reps}


def host_path_bench(db, sel_host, n, r, q, steps, pir):
    """The synchronous host calls (selection upload, scan, answer download),
    with pageable and with pinned (pir_host_alloc) buffers: PCIe-inclusive
    rates, reported beside the resident-input figures, never in their place."""
    import numpy as np
    row = (n + 7) // 8
    res = {"steps": steps, "sel_bytes_per_query": row}
    for qq in (1, q):
        src = sel_host[:qq, :row]  # host pitch = ceil(N/8): one contiguous upload per query
        page_sel = np.ascontiguousarray(src)
        page_out = np.empty((qq, r), np.uint8)
        pin_sel = pir.pinned_empty((qq, row))
        pin_sel[:] = src
        pin_out = pir.pinned_empty((qq, r))
        entry = {}
        for name, a, o in (("pageable", page_sel, page_out), ("pinned", pin_sel, pin_out)):
            db.dpxor_batch(a, out=o)  # warm-up: staging buffers, plan, graph
            t = time.perf_counter()
            for _ in range(steps):
                db.dpxor_batch(a, out=o)
            ms = (time.perf_counter() - t) / steps * 1e3
            entry[name] = {"ms_per_call": ms, "queries_per_s": qq / ms * 1e3,
                           "sel_gbs": qq * row / (ms / 1e3) / 1e9}
        assert np.array_equal(pin_out, page_out)
        res[f"q{qq}"] = entry
        log(f"host path Q={qq}: pageable {entry['pageable']['ms_per_call']:.2f} ms, "
            f"pinned {entry['pinned']['ms_per_call']:.2f} ms per call")
        del pin_sel, pin_out
    return res


def dpf_bench(ctx, db, db_host, n, r, args, torch, pir):
    """DPF evaluation on the database's domain and answers straight from keys."""
    import numpy as np
    import synth

    nb = pir.dpf_domain_bits(n)
    nk = args.dpf_keys
    rng = np.random.default_rng(11)
    alphas = [int(a) for a in rng.integers(0, n, nk // 2)]
    keys = []
    for i, a in enumerate(alphas):
        root = synth.stream_bytes(synth.S_KEY + 900 + i, 32)
        k0, k1 = pir.dpf_gen(a, nb, root[:16], root[16:])
        keys += [k0, k1]
    d_keys = torch.from_numpy(np.stack(keys)).to("cuda:0")
    words = (n + 31) // 32
    d_sel = torch.empty((nk, words), dtype=torch.int32, device="cuda:0")

    def step_eval():
        ctx.dpf_eval_async(d_keys, nb, nk, n, d_sel)

    for _ in range(2):
        step_eval()
    torch.cuda.synchronize()
    ctx.timing(True)
    ctx.timing_read(reset=True)
    wall, _ = time_steps(step_eval, args.dpf_steps, torch)
    t = ctx.timing_read(reset=True)
    ctx.timing(False)
    ms = t["dpf_ms"] / max(1, t["dpf_evals"])
    # Eval(k0) XOR Eval(k1) is the indicator of alpha
    ok = True
    for i, a in enumerate(alphas):
        x = d_sel[2 * i] ^ d_sel[2 * i + 1]
        nz = torch.nonzero(x).flatten().cpu().tolist()
        ok &= nz == [a // 32] and (int(x[a // 32].item()) & 0xFFFFFFFF) == 1 << (a % 32)
    half = 1 << (nb - 1) if nb else 0
    ops = ((half - 1) * DPF_OPS_FULL + half * DPF_OPS_LEAF) * nk if n == 1 << nb else None
    out = {
        "domain_bits": nb, "keys_per_call": nk, "ms_per_call": ms, "ms_per_key": ms / nk,
        "leaves_per_s": nk * n / (ms / 1e3), "node_expansions_per_s": nk * ((1 << nb) - 1) / (ms / 1e3),
        "point_function_check": bool(ok),
    }
    if ops is not None:
        ach = ops / (ms / 1e3) / 1e12
        out["roofline"] = {"bound": "alu", "achieved": ach, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                           "frac": ach / VALU_PEAK_TOPS, "traffic": None,
                           "algorithmic_ops_per_launch": ops, "avg_launch_ms": ms,
                           "ops_per_expansion": {"full": DPF_OPS_FULL, "leaf": DPF_OPS_LEAF}}
    log(f"DPF eval: {ms / nk:.3f} ms per key (2^{nb} leaves), point check {ok}")

    # answers from keys: evaluation into a workspace, then the batched scan
    d_ans = torch.empty((nk, r), dtype=torch.uint8, device="cuda:0")

    def step_answer():
        db.dpf_dpxor_async(d_keys, nk, d_ans)

    step_answer()
    torch.cuda.synchronize()
    wall_a, _ = time_steps(step_answer, args.dpf_steps, torch)
    ans = d_ans.cpu().numpy()
    ok_a = all(np.array_equal(ans[2 * i] ^ ans[2 * i + 1], db_host[a]) for i, a in enumerate(alphas))
    out["key_to_answer"] = {"queries_per_s": nk * args.dpf_steps / wall_a,
                            "ms_per_call": wall_a / args.dpf_steps * 1e3, "two_server_check": bool(ok_a)}
    log(f"keys -> answers: {out['key_to_answer']['queries_per_s']:.1f} q/s, two-server check {ok_a}")

    if args.cpu_sample > 0:
        out["cpu_baseline"] = dpf_cpu_baseline(keys[0])
    return out


def dpf_cpu_baseline(key_full_domain):
    """The oracle's DPF evaluation, one host thread, on a 2^16-leaf domain."""
    import numpy as np
    import oracle
    import paper_2509_06514_amd as pir
    import synth

    nb = 16
    root = synth.stream_bytes(synth.S_KEY + 999, 32)
    k0, _ = pir.dpf_gen(12345, nb, root[:16], root[16:])
    t0 = time.perf_counter()
    oracle.dpf_eval_full(k0, nb)
    dt = time.perf_counter() - t0
    return {"value": (1 << nb) / dt, "unit": "leaves/s", "cores": 1, "kind": "oracle",
            "sample": f"one key over 2^{nb} leaves (each leaf evaluated root to leaf, as eq. 1-3 "
                      f"read), {dt:.2f} s on 1 host thread"}


FP_SHAPE = (1 << 24, 32, 127)  # records, elements per record, p


def fp_bench(ctx, args, torch, pir):
    """Inner products over F_p on the int8 matrix cores (HBM-bound scan)."""
    import numpy as np
    import synth

    n, L, p = FP_SHAPE
    q = args.fp_queries
    D = (synth.stream_bytes(synth.S_DB + 9, n * L).reshape(n, L) % p).astype(np.uint8)
    db = ctx.load_fp_db(D, p)
    stride = db.v_stride  # recommended pitch: an odd multiple of 128 bytes
    rows = (synth.stream_bytes(synth.S_SEL + 9, q * stride).reshape(q, stride) & 127).astype(np.uint8)
    # rows 0 and 1: additive shares of the unit vector at index i
    i = n // 3
    e = np.zeros(stride, np.int64)
    e[i] = 1
    rows[1] = ((e - (rows[0] % p)) % p).astype(np.uint8)
    rows[:, n:] = 0
    d_v = torch.from_numpy(rows).to("cuda:0")
    d_out = torch.empty((q, L), dtype=torch.uint8, device="cuda:0")
    out = {"n_records": n, "record_elems": L, "p": p, "q": q, "v_stride": stride}
    for qq in (q, 1):
        def step():
            db.inner_async(d_v, qq, d_out)
        for _ in range(3):
            step()
        torch.cuda.synchronize()
        # passes timed with the library's kernel timing off (its events add
        # work between launches), then the kernel durations in a pass of their own
        wall, per = time_steps(step, args.steps, torch)
        ctx.timing(True)
        ctx.timing_read(reset=True)
        time_steps(step, max(3, min(args.steps, 10)), torch)
        t = ctx.timing_read(reset=True)
        ctx.timing(False)
        s1 = t["fp_ms"] / max(1, t["fp_launches"])
        alg = n * L + qq * db.min_v_stride + qq * L
        ach = alg / (s1 / 1e3) / 1e9
        rec = {"ms_per_pass": wall / args.steps * 1e3, "queries_per_s": qq * args.steps / wall,
               "latency_ms": {"p50": percentile(per, 0.5), "p99": percentile(per, 0.99)},
               "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": ach / HBM_PEAK_GBS, "traffic": load_fp_traffic(qq, L),
                            "algorithmic_bytes_per_launch": alg,
                            "avg_launch_ms": s1}}
        if qq == q:
            out.update(rec)
            ans = d_out.cpu().numpy()
            out["two_server_check"] = bool(np.array_equal((ans[0].astype(int) + ans[1]) % p, D[i]))
        else:
            out["single_query"] = rec
        log(f"F_p q={qq}: stage1 {s1:.3f} ms, {ach:.0f} GB/s")
    if args.cpu_sample > 0:
        import oracle
        t0 = time.perf_counter()
        oracle.fp_inner(D, rows[0][:n], p)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 1.0 / dt, "unit": "queries/s", "cores": 1, "kind": "oracle",
                               "sample": f"1 query over N={n} records of {L} elements (p={p}) on 1 host thread, "
                                         f"{dt:.2f} s"}
    db.free()
    return out


def load_fp_traffic(q, L):
    """HBM bytes per launch of the F_p stage-1 kernel from the committed counter runs, if they are
    for this source and kernel instance; else None."""
    try:
        with open(os.path.join(ROOT, "profiles", "traffic_fp_n24.json")) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    entry = t.get(f"q{q}")
    if not entry or t.get("kernel_source_sha256_16") != kernel_source_hash("pir_fp.hip"):
        return None
    rt = 1 if q <= 16 else 2 if q <= 32 else 4
    n_ct = (L + 15) // 16
    ct = 4 if n_ct >= 4 else 2 if n_ct >= 2 else 1
    if entry.get("kernel") != f"k_fp_stage1_lds<{rt}, {ct}>":
        return None
    return entry.get("hbm_bytes_per_launch")


SERVE_DBS = [(1 << 23, 32), (1 << 24, 128), (1 << 22, 1024)]


def serve_bench(args):
    """Open-loop Poisson arrivals over three resident databases (continuous batching).

    Each rate runs for at least 10 s or 20k requests (and at least
    args.serve_seconds); each request goes to a database drawn uniformly;
    selections come from a pool of 16 per database (contents do not change the
    scan's cost).  Latency is submit -> answer in host memory, measured by the
    server.  After each rate, the last answer written to every output slot is
    compared with the same selection answered alone by the library's
    synchronous call ("alone vs in the mix").
    """
    import threading

    import numpy as np

    import synth
    import paper_2509_06514_amd as pir

    # submitters sleep until their next arrival (no spinning) and hand the
    # interpreter lock on quickly, so arrivals are not bunched by the lock
    sys.setswitchinterval(100e-6)
    ctx = pir.Context(0)
    hosts, dbs = [], []
    for k, (n, r) in enumerate(SERVE_DBS):
        h = synth.database(n, r, seed=synth.S_DB + 5 + k)
        dbs.append(ctx.load_db(h))
        hosts.append(h)
        log(f"serve: loaded DB{k} N={n} R={r}")
    # tune every batch-size bucket (powers of two up to q_max) the server can form
    for k, d in enumerate(dbs):
        qq = 1
        while True:
            d.tune(min(qq, args.serve_qmax))
            if qq >= args.serve_qmax:
                break
            qq *= 2
        log(f"serve: tuned DB{k} for batches of 1 .. {args.serve_qmax}")
    pool = [synth.selections(n, 16, seed=synth.S_SEL + 50 + k) for k, (n, r) in enumerate(SERVE_DBS)]
    alone = [d.dpxor_batch(p) for d, p in zip(dbs, pool)]  # each pool row answered on its own call
    if args.serve_keys:
        # requests are DPF keys: a pool per database (the server's cost does not
        # depend on alpha), plus one key pair per database checked afterwards
        kpool, checks = [], []
        for k, (n, r) in enumerate(SERVE_DBS):
            nb = pir.dpf_domain_bits(n)
            keys = []
            for j in range(16):
                root = synth.stream_bytes(synth.S_KEY + 100 * k + j, 32)
                keys.append(pir.dpf_gen((j * 7919) % n, nb, root[:16], root[16:])[j % 2])
            kpool.append(keys)
            root = synth.stream_bytes(synth.S_KEY + 100 * k + 99, 32)
            checks.append((n // 2,) + pir.dpf_gen(n // 2, nb, root[:16], root[16:]))
    results = []
    rates = [int(x) for x in (args.serve_key_rates if args.serve_keys else args.serve_rates).split(",")]
    threads_n = args.serve_threads
    slots_per_thread = 512
    for rate in rates:
        srv = pir.Server(ctx, q_max=args.serve_qmax, max_wait_us=args.serve_wait_us, n_slots=args.serve_slots,
                         queue_cap=1 << 20)
        ids = [srv.add_db(d) for d in dbs]
        outs = [np.zeros((threads_n * slots_per_thread, r), np.uint8) for (n, r) in SERVE_DBS]
        last = [np.full(threads_n * slots_per_thread, -1, np.int64) for _ in SERVE_DBS]  # pool row last written
        # at least 10 s or 20k requests per rate (whichever comes first), at least serve_seconds
        dur = min(10.0, max(args.serve_seconds, 20000.0 / rate))
        stop_at = time.perf_counter() + dur
        pending = [[] for _ in range(threads_n)]
        rejected = [0] * threads_n

        def submitter(tid):
            rng = np.random.default_rng(1000 * rate + tid)
            t = time.perf_counter()
            k = 0
            lib_submit = srv.submit_key_raw if args.serve_keys else srv.submit_raw
            while True:
                t += rng.exponential(threads_n / rate)
                if t > stop_at:
                    break
                dt = t - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                w = int(rng.integers(0, 3))
                src = kpool[w][k % 16] if args.serve_keys else pool[w][k % 16]
                slot = tid * slots_per_thread + k % slots_per_thread
                out = outs[w][slot]
                rc, tk = lib_submit(ids[w], src.ctypes.data, out.ctypes.data)
                if rc == 0:
                    pending[tid].append(tk)
                    last[w][slot] = k % 16
                else:
                    rejected[tid] += 1
                k += 1

        ths = [threading.Thread(target=submitter, args=(i,)) for i in range(threads_n)]
        clock = []
        clock_stop = threading.Event()
        if args.serve_clock_ms > 0:
            ths_clock = threading.Thread(target=sample_engine_clock,
                                         args=(args.serve_clock_ms / 1e3, clock_stop, clock), daemon=True)
        srv.stats(reset=True)
        if args.serve_clock_ms > 0:
            ths_clock.start()
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        if args.serve_clock_ms > 0:
            clock_stop.set()
            ths_clock.join()
        for lst in pending:
            for tk in lst:
                srv.wait(tk, 60000)
        st = srv.stats()
        check = None
        if args.serve_keys:
            # the two parties' answers for one index per database reconstruct the record
            check = True
            for w, (alpha, k0, k1) in enumerate(checks):
                a0, a1 = np.zeros(SERVE_DBS[w][1], np.uint8), np.zeros(SERVE_DBS[w][1], np.uint8)
                t0k, t1k = srv.submit_key(ids[w], k0, a0), srv.submit_key(ids[w], k1, a1)
                check &= srv.wait(t0k, 60000) == 0 and srv.wait(t1k, 60000) == 0
                check &= bool(np.array_equal(a0 ^ a1, hosts[w][alpha]))
        srv.close()
        hist = {f"{1 << i}-{(2 << i) - 1}": c for i, c in enumerate(st["batch_hist"]) if c}
        rec = {"offered_qps": rate, "seconds": dur, "achieved_qps": st["completed"] / dur,
               "completed": st["completed"], "rejected": st["rejected"] + sum(rejected),
               "blocked_submits": st["blocked_submits"],
               "p50_ms": st["p50_us"] / 1e3, "p99_ms": st["p99_us"] / 1e3, "mean_ms": st["mean_us"] / 1e3,
               "max_ms": st["max_us"] / 1e3,
               "batches": st["batches"], "batch_hist": hist, "max_inflight": st["max_inflight"],
               "h2d_GBps": st["h2d_bytes"] / dur / 1e9}
        if clock:
            cs = sorted(clock)
            rec["engine_clock_mhz"] = {"samples": len(cs), "median": cs[len(cs) // 2], "p10": cs[len(cs) // 10],
                                       "p90": cs[9 * len(cs) // 10], "min": cs[0],
                                       "below_500": sum(1 for c in cs if c < 500) / len(cs)}
        if check is not None:
            rec["two_server_check"] = bool(check)
        else:
            checked = same = 0
            for w in range(3):
                for slot in np.nonzero(last[w] >= 0)[0]:
                    checked += 1
                    same += bool(np.array_equal(outs[w][slot], alone[w][last[w][slot]]))
            rec["answers_checked_vs_alone"] = checked
            rec["answers_same_as_alone"] = same == checked
        log(f"serve rate {rate}: {json.dumps(rec)}")
        results.append(rec)
    for d in dbs:
        d.free()
    ctx.close()
    return results


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # the first 10-20 scan replays after tuning run slower (the scan's clock
    # is still settling: 35.6-36.0 k q/s over 20 steps after 3 warm-up steps,
    # 37.4-37.7 k q/s after 30, on the same machine); warm-up steps are untimed
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--config", default="n28r32q64", choices=sorted(CONFIGS))
    ap.add_argument("--no-tune", action="store_true", help="use the default kernel plan")
    ap.add_argument("--variants", action="store_true",
                    help="also time the best plan of each kernel family (VALU, int8 MFMA, fp4 MFMA) for Q")
    ap.add_argument("--cpu-sample", type=int, default=2, help="oracle queries for cpu_baseline (0 = skip)")
    ap.add_argument("--cpu-threads", type=int, default=affinity_threads(),
                    help="host threads for the all-core oracle baseline (one query each; default: every "
                         "thread this process may run on)")
    ap.add_argument("--sel-fill", default="random", choices=["random", "zeros", "ones"],
                    help="selection contents (zeros/ones: the scan must read the same bytes)")
    ap.add_argument("--serve-keys", action="store_true", help="serving sweep with DPF keys as requests")
    ap.add_argument("--serve-key-rates", default="500,1000,2000,4000",
                    help="offered rates for --serve-keys (each key costs a full-domain evaluation)")
    ap.add_argument("--no-single", action="store_true", help="skip the single-query pass")
    ap.add_argument("--host-steps", type=int, default=3,
                    help="calls per case of the synchronous host-buffer path (0 = skip)")
    ap.add_argument("--dpf-keys", type=int, default=8,
                    help="DPF keys (pairs of parties) evaluated per call in the DPF section (0 = skip)")
    ap.add_argument("--dpf-steps", type=int, default=5)
    ap.add_argument("--fp-queries", type=int, default=64,
                    help="queries per pass in the F_p inner-product section (0 = skip)")
    ap.add_argument("--serve", action="store_true", help="run the serving sweep (three resident DBs) instead")
    ap.add_argument("--serve-rates", default="1000,2000,5000,10000,20000,50000")
    ap.add_argument("--serve-seconds", type=float, default=3.0)
    ap.add_argument("--serve-threads", type=int, default=8)
    ap.add_argument("--serve-qmax", type=int, default=64)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-wait-us", type=int, default=200)
    ap.add_argument("--serve-clock-ms", type=float, default=0.0,
                    help="sample the engine clock (sysfs pp_dpm_sclk) every this many ms while serving; "
                         "the polling itself can change the device's power states")
    ap.add_argument("--no-read-roof", action="store_true", help="skip the streaming-read roof probe")
    ap.add_argument("--phase-steps", type=int, default=10,
                    help="rounds of the per-phase breakdown (selection upload, stages, answer download; 0 = skip)")
    ap.add_argument("--calib-copy-gib", type=int, default=0,
                    help="first run a plain device copy of this many GiB, 3 times (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(across GPUs the scan would shard by queries or by record ranges)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2509_06514_amd as pir

    if args.serve:
        res = serve_bench(args)
        print(json.dumps({"metric": "serving p50/p99 latency vs offered load (3 resident DBs"
                                    + (", requests as DPF keys)" if args.serve_keys else ")"),
                          "unit": "ms", "data": "synthetic",
                          "config": {"dbs": [{"n_records": n, "record_bytes": r} for n, r in SERVE_DBS],
                                     "q_max": args.serve_qmax, "slots": args.serve_slots,
                                     "max_wait_us": args.serve_wait_us,
                                     "seconds_per_rate": "max(serve_seconds, min(10, 20000 / rate))"},
                          "rates": res}), flush=True)
        return

    if args.calib_copy_gib > 0:
        # a plain copy kernel of known size: reads and writes calib_copy_gib GiB per launch
        nbytes = args.calib_copy_gib << 30
        a = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy: 3 x {nbytes} bytes")
        del a, b

    n, r, q = CONFIGS[args.config]
    log(f"config {args.config}: N={n} R={r} Q={q}")
    t = time.perf_counter()
    db_host = synth.database(n, r, seed=synth.S_DB + 3)
    log(f"generated {n * r / 2**30:.2f} GiB database in {time.perf_counter() - t:.1f}s")
    stride = pir.sel_stride_for(n)
    sel_host = synth.selections(n, q, seed=synth.S_SEL + 3, stride=stride)
    if args.sel_fill != "random":
        sel_host[:] = 0 if args.sel_fill == "zeros" else 0xFF

    ctx = pir.Context(0)
    roof = None if args.no_read_roof else read_roof(ctx, n * r, torch)
    t = time.perf_counter()
    db = ctx.load_db(db_host)
    log(f"loaded into HBM in {time.perf_counter() - t:.1f}s")
    dev = torch.device("cuda:0")
    d_sel = torch.from_numpy(sel_host).to(dev)
    d_out = torch.empty((q, r), dtype=torch.uint8, device=dev)
    d_out1 = torch.empty((1, r), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    log(f"{'planning' if args.no_tune else 'tuning'} Q={q} ...")
    cfg_q = db.get_cfg(q) if args.no_tune else db.tune(q)
    cfg_1 = None
    if not args.no_single:
        log(f"{'planning' if args.no_tune else 'tuning'} Q=1 ...")
        cfg_1 = db.get_cfg(1) if args.no_tune else db.tune(1)
    log(f"plan Q={q}: {cfg_q}; plan Q=1: {cfg_1}")

    step_q = lambda: db.dpxor_batch_async(d_sel, q, d_out, sel_stride=stride)  # noqa: E731
    step_1 = lambda: db.dpxor_batch_async(d_sel, 1, d_out1, sel_stride=stride)  # noqa: E731

    for _ in range(args.warmup):
        step_q()
        if not args.no_single:
            step_1()
    torch.cuda.synchronize()

    # timed: K batched steps, each one replay of the scan's captured hipGraph
    wall_q, per_q = time_steps(step_q, args.steps, torch)
    # kernel durations: the same steps with the library's HIP events around each
    # stage (launches enqueued one by one while timing is on)
    n_timed = max(3, min(args.steps, 10))
    ctx.timing(True)
    ctx.timing_read(reset=True)
    time_steps(step_q, n_timed, torch)
    tq = ctx.timing_read(reset=True)
    ctx.timing(False)
    log(f"Q={q}: {wall_q / args.steps * 1e3:.3f} ms/step, stage1 avg "
        f"{tq['stage1_ms'] / max(1, tq['stage1_launches']):.3f} ms, stage2 avg "
        f"{tq['stage2_ms'] / max(1, tq['stage2_launches']):.4f} ms")

    single = None
    if not args.no_single:
        wall_1, per_1 = time_steps(step_1, args.steps, torch)
        ctx.timing(True)
        ctx.timing_read(reset=True)
        time_steps(step_1, n_timed, torch)
        t1 = ctx.timing_read(reset=True)
        ctx.timing(False)
        s1_avg = t1["stage1_ms"] / max(1, t1["stage1_launches"])
        ms1 = wall_1 / args.steps * 1e3
        single = {
            "ms_per_query": ms1,
            "queries_per_s": 1e3 / ms1,
            "db_gbs_scanned": n * r / (ms1 / 1e3) / 1e9,
            "latency_ms": {"p50": percentile(per_1, 0.5), "p99": percentile(per_1, 0.99)},
            "cfg": cfg_1.as_dict(),
            "roofline": roofline_for(cfg_1.variant, n, r, 1, s1_avg, load_traffic(n, r, 1, cfg_1),
                                     roof["achieved_gbs"] if roof else None),
        }
        log(f"Q=1: {ms1:.3f} ms/query, {single['db_gbs_scanned']:.0f} GB/s scanned, stage1 avg {s1_avg:.3f} ms")

    ms_step = wall_q / args.steps * 1e3
    qps = q * args.steps / wall_q
    s1q = tq["stage1_ms"] / max(1, tq["stage1_launches"])
    result = {
        "metric": "DB GB/s scanned & queries/s (1 vs Q=64 batched) at 8 GiB; p50/p99 latency",
        "value": qps,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": VARIANT_DTYPE.get(cfg_q.variant, "u32"),
        "data": "synthetic",
        "config": {"workload": f"dpXOR, N={n} records x {r} B ({n * r / 2**30:.0f} GiB), Q={q} "
                               "selection vectors answered in one database pass per step",
                   "n_records": n, "record_bytes": r, "q": q, "global_batch": q,
                   "parallelism": "single GPU", "kernel_cfg": cfg_q.as_dict(),
                   "launch": "hipGraph replay (stage 1 + stage 2)"},
        "db_gbs_scanned": n * r / (ms_step / 1e3) / 1e9,
        "latency_ms": {"p50": percentile(per_q, 0.5), "p99": percentile(per_q, 0.99)},
        "stage_ms": {"stage1_avg": s1q, "stage2_avg": tq["stage2_ms"] / max(1, tq["stage2_launches"])},
        "roofline": roofline_for(cfg_q.variant, n, r, q, s1q, load_traffic(n, r, q, cfg_q),
                                 roof["achieved_gbs"] if roof else None),
    }
    if roof:
        result["read_roof"] = roof
    if single is not None:
        result["single_query"] = single
        result["batched_vs_single_qps"] = qps / single["queries_per_s"]

    # this run's answers, compared with the oracle's rows when cpu_baseline runs
    ans = d_out.cpu().numpy()
    result["answers_nonzero"] = bool(ans.any())

    if args.phase_steps > 0:
        result["phases"] = phase_breakdown(ctx, db, sel_host, stride, r, [1, q] if q > 1 else [1],
                                           args.phase_steps, torch)

    if args.host_steps > 0:
        result["host_path"] = host_path_bench(db, sel_host, n, r, q, args.host_steps, pir)

    if args.variants:
        result["variants"] = variant_sweep(ctx, db, d_sel, stride, n, r, q, d_out, torch, pir)

    if args.dpf_keys > 0:
        result["dpf"] = dpf_bench(ctx, db, db_host, n, r, args, torch, pir)

    if args.fp_queries > 0:
        result["fp"] = fp_bench(ctx, args, torch, pir)

    if args.cpu_sample > 0:
        log(f"cpu_baseline: oracle on {args.cpu_sample} queries ...")
        rec, want = cpu_baseline(db_host, sel_host, n, r, args.cpu_sample, args.cpu_threads)
        result["cpu_baseline"] = rec
        k = min(q, want.shape[0])
        bad = [i for i in range(k) if not np.array_equal(ans[i], want[i])]
        result["oracle_rows_match"] = {"rows_checked": k, "match": not bad, "mismatched_rows": bad[:16]}
        log(f"oracle rows 0..{k - 1}: {'all match' if not bad else f'{len(bad)} differ'}")
    else:
        result["cpu_baseline"] = None

    db.free()
    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
