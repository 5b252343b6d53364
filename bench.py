#!/usr/bin/env python3
"""Benchmark of the semiring closure hot path on one MI355X.

Default workload (the headline): anti-distance Floyd-Warshall closure of a
D = 8192 uint16 random digraph (edge probability 0.05, distances uniform in
[1, 1000], 1% of edges with distances in [64536, 65534]).  One step = one full
closure (all three phases of every round) of a fresh copy of the input that is
already resident in HBM.  Metric: semiring updates per second, D^3 / t.

Other workloads (--workload): bool16384 (Boolean closure, D = 16384, mean
out-degree 3 plus planted strongly connected blocks), boolmul16384 (Boolean
product A * A of that matrix, word-parallel and int8 matrix-core paths),
mul1024 (uint16 product of two 1024 x 1024 graphs), small (latencies of the
Boolean 256-vertex product and closure and the uint16 1024-vertex product and
closure), u8fw8192 (uint8 closure,
distances in [1, 200]), dfw8192 (the headline input as a distance matrix,
closed with min and saturating +), u32fw8192 (the headline distances in
uint32 entries, S = 2^32 - 1), batched (4096 graphs, log-uniform sizes in
[32, 1024], uint16: the prepared batch with autotuned update tiles replayed as
one graph launch, vs one closure_batched call and vs one closure per graph;
then the same batch as uint8), add8192 (entrywise max, HBM-bound), serve
(continuously batched closure requests vs serial).

Prints one JSON line.  The roofline object is for the dominant kernel (the
update phase), timed live with hipEvents on its own stream; cpu_baseline is
the oracle's Warshall loop on a bounded sample of the same input.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 64 VALU lanes x 2.4 GHz = 3.93e13 32-bit lane operations
# per second; one packed saturating-subtract + one packed max cover two
# anti-distance updates, i.e. one lane operation per update.  A v_bitop3_b32
# covers 32 Boolean updates.  HBM peak 8 TB/s.
VALU_LANE_OPS = 256 * 64 * 2.4e9
PEAK_ANTIDIST = VALU_LANE_OPS
# uint8 data are held as binary16 values: two inner steps of a packed pair are
# two v_pk_add_f16 and one v_pk_maximum3_f16 (0.75 lane operations per update)
PEAK_ANTIDIST_U8 = VALU_LANE_OPS / 0.75
# uint32 entries are not packed: a saturating subtract per update, and one
# v_max3_u32 per two updates (1.5 lane operations per update)
PEAK_ANTIDIST32 = VALU_LANE_OPS / 1.5
PEAK_BOOL = 32 * VALU_LANE_OPS
# dense int8 matrix-core rate (MI355X datasheet: 5.0 POP/s = 2.5e15 MAC/s); one
# MAC is one Boolean update on the SR_BOOL_MFMA path
PEAK_I8_MAC = 2.5e15
# dense fp4 matrix-core rate (MI355X datasheet: 10.1 PFLOP/s = 5.05e15 MAC/s)
PEAK_F4_MAC = 5.05e15

# HBM traffic of the update kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE,
# scaled by the same counters on a streaming kernel of known size; valid only
# for the kernel sources whose hash is recorded with it (None until measured).
TRAFFIC = {
    # full update launch (252 x 32 workgroups, every tile outside the pivot
    # row and column blocks) of the D = 8192 closure:
    # FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000, in bytes
    "fw8192": {"src_hash": "f8d45de227bbaa9f", "bytes_per_launch": 4.974e8},   # 1.794e5 + 1.270e5 KiB
    "u8fw8192": {"src_hash": "f8d45de227bbaa9f", "bytes_per_launch": 4.841e8},  # 1.729e5 + 1.270e5 KiB
    "dfw8192": {"src_hash": "f8d45de227bbaa9f", "bytes_per_launch": 4.970e8},  # 1.792e5 + 1.270e5 KiB
    "u32fw8192": {"src_hash": "c4166400949ed0ba", "bytes_per_launch": 7.185e8},  # 2.219e5 + 2.579e5 KiB
    # full update launches (matrix-core kernel, 4-bit operands) of the
    # serialized D = 16384 Boolean closure
    "bool16384": {"src_hash": "1b38e735282477e3", "bytes_per_launch": 7.014e7},  # 1.836e4 + 3.178e4 KiB
}


def src_hash(workload):
    """Hash of the device source of the workload's update kernel: for
    anti-distance the tile code (sr_tiles.h but the pivot tile's closure) and
    the text of the k_ad_fw_update kernel template (host-side changes
    elsewhere in sr_antidist.hip do not change the kernel); for Boolean
    the device code of sr_bool_mfma.hip (the matrix-core update); for
    the uint32 path the update kernel's text and the device code before the
    product kernel in sr_antidist32.hip."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1705_08743_amd/csrc")
    if workload.startswith("bool"):
        # the device code of sr_bool_mfma.hip (it ends where the host-side
        # launch helpers begin)
        with open(os.path.join(csrc, "sr_bool_mfma.hip")) as f:
            text = f.read()
        h.update(text[:text.index("// Operand format of the matrix-core path")].encode())
        return h.hexdigest()[:16]
    if workload.startswith("u32"):
        # the update kernel and the device code it runs (the step functions,
        # the wave tiles), not the product kernel or the host side
        with open(os.path.join(csrc, "sr_antidist32.hip")) as f:
            text = f.read()
        a = text.index("__device__ __forceinline__ uint32_t step32(")
        b = text.index("// Product: grid (column chunks")
        c = text.index("k_ad32_update(uint32_t *T")
        d = text.index("\n}\n", c)
        h.update(text[a:b].encode())
        h.update(text[c:d].encode())
        return h.hexdigest()[:16]
    # the tile code the update kernel runs (sr_tiles.h without the pivot
    # tile's closure) and the update kernel's own text
    with open(os.path.join(csrc, "sr_tiles.h")) as f:
        tiles = f.read()
    a = tiles.rfind("// ----", 0, tiles.index("// Warshall closure of one bs x bs tile"))
    b = tiles.index("// Number of phase-2 workgroups of a round:")
    h.update((tiles[:a] + tiles[b:]).encode())
    with open(os.path.join(csrc, "sr_antidist.hip")) as f:
        text = f.read()
    start = text.index("k_ad_fw_update(uint16_t *T")
    end = text.index("\n}\n", start)
    h.update(text[start:end].encode())
    return h.hexdigest()[:16]


def traffic_of(workload):
    tr = TRAFFIC.get(workload, {})
    ok = tr.get("src_hash") is not None and tr.get("src_hash") == src_hash(workload)
    return tr.get("bytes_per_launch") if ok else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sync_all(torch):
    if torch.distributed.is_available() and torch.distributed.is_initialized():
        torch.distributed.barrier()
    torch.cuda.synchronize()


def oracle_threads():
    """Threads the oracle may use: the CPUs this process may run on, capped
    by OMP_NUM_THREADS when the machine sets it (a share of a larger host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def host_cpu():
    """The host CPU the oracle runs on: model name, logical CPUs of the
    machine, CPUs this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = os.cpu_count() or 1
    return {"model": model, "logical_cpus": os.cpu_count(), "cpus_allowed": allowed,
            "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS")}


def oracle_fw(A, S, dual, threads):
    """The oracle's whole Warshall loop on the input (distance loop for
    distance matrices), on `threads` threads: (result, seconds)."""
    import oracle
    oracle.set_threads(threads)
    t0 = time.perf_counter()
    want = oracle.dist_closure(A, S) if dual else oracle.ad_closure(A, S)
    return want, time.perf_counter() - t0


def oracle_fw_one_thread(A, S, dual, target_s):
    """The oracle's loop on one thread over the first m pivots of the same
    input (m sized to about target_s seconds): updates/s and the sample."""
    import numpy as np
    import oracle
    oracle.set_threads(1)
    D = A.shape[0]
    if dual:
        # the distance loop has no prefix entry point; its anti-distance twin
        # on the complemented input does the same work per pivot
        A = (S - A.astype(np.int64))
    A = np.ascontiguousarray(A, dtype=np.int64 if S > 2 ** 31 - 1 else np.int32)
    m0 = min(D, 4)
    t0 = time.perf_counter()
    oracle.ad_closure(A, S, k_end=m0)
    t1 = time.perf_counter()
    oracle.ad_closure(A, S, k_end=2 * m0)
    t2 = time.perf_counter()
    per_pivot = max((t2 - t1) - (t1 - t0), 1e-9) / m0
    m = int(max(m0, min(D, target_s / per_pivot)))
    t0 = time.perf_counter()
    oracle.ad_closure(A, S, k_end=m)
    dt = time.perf_counter() - t0
    upd = float(m) * D * D
    return upd / dt, ("first %d of %d Warshall pivots of the same input on 1 thread "
                      "(%.3g updates, %.1f s)" % (m, D, upd, dt))


def arena_mats(arena, dtype):
    """Host copies of every matrix of a BatchArena (one device-to-host copy)."""
    import numpy as np
    img = arena.buf.cpu().numpy()
    es = np.dtype(dtype).itemsize
    out = []
    for i in range(arena.count):
        n, ld, off = int(arena.sizes[i]), int(arena.lds[i]), int(arena.offsets[i])
        w = -(-n // 64) if dtype == np.uint64 else n
        out.append(img[off:off + n * ld * es].view(dtype).reshape(n, ld)[:, :w])
    return out


def oracle_batch_parity(got, mats, close):
    """Every graph of a batch against the oracle (close(m) -> its closure):
    (graphs that differ, seconds the oracle took)."""
    import numpy as np
    bad = 0
    t = 0.0
    for g, m in zip(got, mats):
        t0 = time.perf_counter()
        want = close(m)
        t += time.perf_counter() - t0
        if not np.array_equal(g.astype(want.dtype), want):
            bad += 1
    return bad, t


def kernel_timing_pass(args, torch, sr, kind, src, bufs, close):
    """Per-phase launch durations (hipEvents on the launching stream) over
    `steps` closures run with serialized phases; returns ms, launches, avg
    and the algorithmic updates per launch for each phase."""
    for b in bufs:
        b.copy_(src)
    sync_all(torch)
    for ph in (sr.SR_PHASE_PIVOT, sr.SR_PHASE_PANELS, sr.SR_PHASE_UPDATE):
        sr.sr_profile_read(kind, ph)  # forget anything recorded earlier
    sr.sr_profile_enable(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        close(bufs[i])
    sync_all(torch)
    t1 = time.perf_counter()
    sr.sr_profile_enable(False)
    phases = {"serial_ms_per_step": (t1 - t0) * 1e3 / args.steps}
    for ph, name in ((sr.SR_PHASE_PIVOT, "pivot"), (sr.SR_PHASE_PANELS, "panels"),
                     (sr.SR_PHASE_UPDATE, "update")):
        ms, n, u = sr.sr_profile_read(kind, ph)
        phases[name] = {"ms_per_step": ms / args.steps, "launches": n,
                        "avg_us": 1e3 * ms / max(n, 1), "updates_per_launch": u / max(n, 1)}
    return phases


def run_fw(args, torch, sr, kind, D, make_input, workload, S, metric, dual=False,
           peak=PEAK_ANTIDIST, kernel="k_ad_fw_update (update phase)"):
    import numpy as np
    log("generating input D=%d ..." % D)
    A = make_input()
    host = np.ascontiguousarray(A[:, :D])
    src = sr.to_device(kind, host)
    bufs = [torch.empty_like(src) for _ in range(max(1, args.steps))]
    warm = torch.empty_like(src)
    for _ in range(args.warmup):
        warm.copy_(src)
        sr.closure(kind, warm)
    for b in bufs:
        b.copy_(src)
    # timed region: the closures as a user runs them (phases overlapped); an
    # event pair on the caller's stream brackets each closure (the closure
    # joins its second stream back into that stream) for the per-step median
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    sync_all(torch)
    t0 = time.perf_counter()
    for i in range(args.steps):
        evs[i][0].record()
        sr.closure(kind, bufs[i])
        evs[i][1].record()
    sync_all(torch)
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    per_step = sorted(a.elapsed_time(b) for a, b in evs)
    ms_median = per_step[len(per_step) // 2]
    # kernel-timing pass: the same closures again with the phases serialized
    # on one stream, each launch bracketed by hipEvents on that stream, so
    # that a launch's duration is its own
    phases = kernel_timing_pass(args, torch, sr, kind, src, bufs, lambda t: sr.closure(
        kind, t, flags=sr.SR_SERIAL_PHASES))
    up = phases["update"]
    achieved = up["updates_per_launch"] / (up["avg_us"] * 1e-6) if up["avg_us"] > 0 else 0.0
    traffic = traffic_of(workload)
    out = {
        "metric": metric,
        "value": float(D) ** 3 / (ms_step * 1e-3),
        "unit": "updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "ms_median_step": ms_median,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {sr.SR_ANTIDIST_U16: "u16", sr.SR_ANTIDIST_U8: "u8",
                  sr.SR_DISTANCE_U16: "u16", sr.SR_ANTIDIST_U32: "u32"}[kind],
        "data": "synthetic",
        "roofline": {"bound": "alu", "kernel": kernel,
                     "achieved": achieved, "peak": peak, "unit": "updates/s",
                     "frac": achieved / peak, "traffic": traffic},
        "phases": phases,
        "fraction_of_valu_roofline_whole_step": float(D) ** 3 / (ms_step * 1e-3) / peak,
    }
    if not args.no_parity or not args.no_cpu_baseline:
        log("the oracle's whole closure on %d host threads ..." % args.cpu_threads)
        want, dt = oracle_fw(host, S, dual, args.cpu_threads)
        if not args.no_parity:
            got = sr.to_host(bufs[-1])
            out["parity"] = {"entries_compared": int(got.size), "whole_matrix": True,
                             "bit_exact": bool(np.array_equal(got.astype(want.dtype), want))}
        del want
        if not args.no_cpu_baseline:
            v1, sample1 = oracle_fw_one_thread(host, S, dual, args.cpu1_seconds)
            out["cpu_baseline"] = {
                "value": float(D) ** 3 / dt, "unit": "updates/s", "cores": args.cpu_threads,
                "kind": "oracle",
                "sample": "the whole closure of the same D=%d input (%.3g updates, %.1f s, "
                          "%d threads)" % (D, float(D) ** 3, dt, args.cpu_threads),
                "seconds": dt, "cpu": host_cpu(),
                "one_thread": {"value": v1, "unit": "updates/s", "sample": sample1}}
    return out


def timed(torch, fn, steps):
    sync_all(torch)
    t0 = time.perf_counter()
    for i in range(steps):
        fn(i)
    sync_all(torch)
    return (time.perf_counter() - t0) * 1e3 / steps


def run_bool(args, torch, sr, synthgen):
    """Boolean closure, D = 16384, bit-packed (32 MiB)."""
    import numpy as np
    import oracle
    D = 16384
    log("generating Boolean input D=%d ..." % D)
    W = synthgen.cfg_bool16384(D=D)
    src = sr.to_device(sr.SR_BOOL, W, cols=D)
    bufs = [torch.empty_like(src) for _ in range(max(1, args.steps))]
    warm = torch.empty_like(src)
    for _ in range(args.warmup):
        warm.copy_(src)
        sr.closure(sr.SR_BOOL, warm, D=D)
    for b in bufs:
        b.copy_(src)
    ms = timed(torch, lambda i: sr.closure(sr.SR_BOOL, bufs[i], D=D), args.steps)
    phases = kernel_timing_pass(args, torch, sr, sr.SR_BOOL, src, bufs, lambda t: sr.closure(
        sr.SR_BOOL, t, D=D, flags=sr.SR_SERIAL_PHASES))
    up = phases["update"]
    achieved = up["updates_per_launch"] / (up["avg_us"] * 1e-6) if up["avg_us"] > 0 else 0.0
    # the D = 16384 Boolean closure compares the bulk update's paths: bit-sliced words,
    # four-Russians tables, and the matrix cores (4-bit float and int8
    # operands); the whole closure (overlapped) and its update launches
    # (serialized phases) for each, every result equal to the default's
    paths = {}
    ref = bufs[-1].clone()
    for name, flags, fmt in (("bitwise", sr.SR_BOOL_BITWISE, None), ("m4r", sr.SR_BOOL_M4R, None),
                             ("mfma_f4", sr.SR_BOOL_MFMA, "f4"), ("mfma_i8", sr.SR_BOOL_MFMA, "i8")):
        if fmt:
            os.environ["SR_MFMA_FORMAT"] = fmt
        for b in bufs:
            b.copy_(src)
        sr.closure(sr.SR_BOOL, warm, D=D, flags=flags)
        t = timed(torch, lambda i: sr.closure(sr.SR_BOOL, bufs[i], D=D, flags=flags), args.steps)
        same = bool(torch.equal(bufs[-1], ref))
        ph = kernel_timing_pass(args, torch, sr, sr.SR_BOOL, src, bufs, lambda x: sr.closure(
            sr.SR_BOOL, x, D=D, flags=flags | sr.SR_SERIAL_PHASES))
        u = ph["update"]
        rate = u["updates_per_launch"] / (u["avg_us"] * 1e-6) if u["avg_us"] > 0 else 0.0
        paths[name] = {"closure_ms": t, "update_avg_us": u["avg_us"], "update_updates_per_s": rate,
                       "equal_to_default": same}
        os.environ.pop("SR_MFMA_FORMAT", None)
    out = {"metric": "semiring updates/s (D³/t) Boolean Warshall closure D=16384",
           "value": float(D) ** 3 / (ms * 1e-3), "unit": "updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bits",
           "data": "synthetic",
           "config": {"workload": "bool_warshall_D16384", "D": D, "mean_out_degree": 3,
                      "planted_scc_blocks": "8 x 512", "pivot_block": 256,
                      "parallelism": "single_gpu"},
           # at this size the update phase runs on the matrix cores with 4-bit
           # float operands (one MAC per nominal bit update); with K = 256
           # inner bits per round a tile's threshold and packing cost more
           # than its MFMAs, so the fraction of the fp4 peak is low although
           # the kernel beats the word kernels (bulk_update_paths)
           "roofline": {"bound": "mfma", "kernel": "k_bool_fw_update_mfma (update phase, fp4)",
                        "achieved": achieved, "peak": PEAK_F4_MAC, "unit": "MAC/s",
                        "frac": achieved / PEAK_F4_MAC, "traffic": traffic_of("bool16384"),
                        "fraction_of_bitwise_peak": achieved / PEAK_BOOL,
                        "note": "nominal D^3 bit updates = MACs; fp4 dense peak 5.05e15 MAC/s; "
                                "bitwise peak one v_bitop3 per 32 updates"},
           "phases": phases, "bulk_update_paths": paths}
    if not args.no_parity or not args.no_cpu_baseline:
        oracle.set_threads(args.cpu_threads)
        t0 = time.perf_counter()
        want = oracle.bool_closure_words(W, D)
        dt = time.perf_counter() - t0
        nw = D // 64
        if not args.no_parity:
            got = sr.to_host(bufs[-1])
            out["parity"] = {"words_compared": int(D * nw), "whole_matrix": True,
                             "bit_exact": bool(np.array_equal(got[:, :nw], want[:, :nw])
                                               and synthgen.padding_bits_clear(got, D))}
        if not args.no_cpu_baseline:
            # one thread: the same whole loop (about 16x the all-threads time)
            oracle.set_threads(1)
            t1 = time.perf_counter()
            oracle.bool_closure_words(W, D)
            dt1 = time.perf_counter() - t1
            oracle.set_threads(args.cpu_threads)
            out["cpu_baseline"] = {
                "value": float(D) ** 3 / dt, "unit": "updates/s", "cores": args.cpu_threads,
                "kind": "oracle",
                "sample": "the whole bit-packed Warshall loop on the same input (%.1f s)" % dt,
                "cpu": host_cpu(),
                "one_thread": {"value": float(D) ** 3 / dt1, "unit": "updates/s",
                               "sample": "the same whole loop on 1 thread (%.1f s)" % dt1}}
    return out


def run_mul(args, torch, sr, synthgen):
    """uint16 product of two 1024 x 1024 graphs (p = 0.05)."""
    import numpy as np
    import oracle
    D = 1024
    A = synthgen.cfg_antidist(D=D, which=0)[:, :D]
    B = synthgen.cfg_antidist(D=D, which=1)[:, :D]
    dA = sr.to_device(sr.SR_ANTIDIST_U16, A)
    dB = sr.to_device(sr.SR_ANTIDIST_U16, B)
    dC = sr.empty(sr.SR_ANTIDIST_U16, D, D)
    f = lambda i: sr.semiring_mul(sr.SR_ANTIDIST_U16, dC, dA, dB)
    for _ in range(args.warmup):
        f(0)
    steps = max(args.steps, 50)
    ms = timed(torch, f, steps)
    out = {"metric": "semiring updates/s (R*K*N/t) anti-distance product 1024^3 uint16",
           "value": float(D) ** 3 / (ms * 1e-3), "unit": "updates/s", "n_gpus": 1,
           "steps": steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u16", "data": "synthetic",
           "config": {"workload": "antidist_u16_product_1024", "R": D, "K": D, "N": D,
                      "parallelism": "single_gpu"},
           "fraction_of_valu_roofline": float(D) ** 3 / (ms * 1e-3) / PEAK_ANTIDIST}
    if not args.no_cpu_baseline or not args.no_parity:
        # the oracle's product of the same two graphs on all host threads:
        # the CPU baseline, and every entry of the parity check
        oracle.set_threads(args.cpu_threads)
        t0 = time.perf_counter()
        want = oracle.ad_mul(A, B, 65535)
        dt = time.perf_counter() - t0
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = {"value": float(D) ** 3 / dt, "unit": "updates/s",
                                   "cores": args.cpu_threads, "kind": "oracle",
                                   "sample": "the whole 1024^3 product", "cpu": host_cpu()}
        if not args.no_parity:
            out["parity"] = {"full_matrix": True, "bit_exact": bool(np.array_equal(
                sr.to_host(dC).astype(np.int64), want))}
    return out


def run_small(args, torch, sr, synthgen):
    """Configurations 1 and 2 as latencies (microseconds per call, median of
    per-call hipEvent pairs): the Boolean D = 256 product A * A and closure,
    the uint16 D = 1024 product A * B and closure."""
    import numpy as np
    import oracle
    W = synthgen.cfg_bool256()
    dW = sr.to_device(sr.SR_BOOL, W, cols=256)
    dWc = sr.clone(dW)
    dP = sr.empty(sr.SR_BOOL, 256, 256)
    A = synthgen.cfg_antidist(D=1024, which=0)[:, :1024]
    B = synthgen.cfg_antidist(D=1024, which=1)[:, :1024]
    dA = sr.to_device(sr.SR_ANTIDIST_U16, A)
    dB = sr.to_device(sr.SR_ANTIDIST_U16, B)
    dAc = sr.clone(dA)
    dC = sr.empty(sr.SR_ANTIDIST_U16, 1024, 1024)
    cases = {
        "bool256_product": (lambda: sr.semiring_mul(sr.SR_BOOL, dP, dW, dW, K=256, N=256), None,
                            256 ** 3),
        "bool256_closure": (lambda: sr.closure(sr.SR_BOOL, dWc, D=256), lambda: dWc.copy_(dW),
                            256 ** 3),
        "u16_1024_product": (lambda: sr.semiring_mul(sr.SR_ANTIDIST_U16, dC, dA, dB), None,
                             1024 ** 3),
        "u16_1024_closure": (lambda: sr.closure(sr.SR_ANTIDIST_U16, dAc), lambda: dAc.copy_(dA),
                             1024 ** 3),
    }
    res = {}
    steps = max(args.steps, 50)
    for name, (fn, reset, upd) in cases.items():
        for _ in range(max(2, args.warmup)):
            if reset:
                reset()
            fn()
        ts = []
        for _ in range(steps):
            if reset:
                reset()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        ts.sort()
        med = ts[len(ts) // 2]
        res[name] = {"us_median": 1e3 * med, "us_min": 1e3 * ts[0], "updates": upd,
                     "updates_per_s": upd / (med * 1e-3)}
    torch.cuda.synchronize()
    out = {"metric": "latency (us per call, median) of the Boolean 256 and uint16 1024 product and closure calls",
           "value": res["u16_1024_closure"]["us_median"], "unit": "us", "n_gpus": 1,
           "steps": steps, "warmup": args.warmup,
           "ms_per_step": res["u16_1024_closure"]["us_median"] * 1e-3,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "u16+bits", "data": "synthetic",
           "config": {"workload": "bool256_and_u16_1024_latency",
                      "parallelism": "single_gpu"},
           "cases": res}
    if not args.no_cpu_baseline:
        # the oracle on the same four calls, one thread and all threads
        cpu = {}
        calls = {"bool256_product": lambda: oracle.bool_mul_words(W, W, 256, 256),
                 "bool256_closure": lambda: oracle.bool_closure_words(W, 256),
                 "u16_1024_product": lambda: oracle.ad_mul(A, B, 65535),
                 "u16_1024_closure": lambda: oracle.ad_closure(A, 65535)}
        for threads in (1, args.cpu_threads):
            oracle.set_threads(threads)
            for name, fn in calls.items():
                t0 = time.perf_counter()
                fn()
                cpu.setdefault(name, {})["ms_%d_threads" % threads] = (time.perf_counter() - t0) * 1e3
        out["cpu_baseline"] = {"value": 1e6 * cpu["u16_1024_closure"]["ms_%d_threads" % args.cpu_threads]
                               / 1e3, "unit": "us", "cores": args.cpu_threads, "kind": "oracle",
                               "sample": "the same four calls, whole (per-call ms in 'calls')",
                               "calls": cpu, "cpu": host_cpu()}
    if not args.no_parity:
        ok = np.array_equal(sr.to_host(dWc)[:, :4], oracle.bool_closure_words(W, 256)[:, :4])
        ok &= np.array_equal(sr.to_host(dP)[:, :4], oracle.bool_mul_words(W, W, 256, 256)[:, :4])
        ok &= np.array_equal(sr.to_host(dC).astype(np.int64), oracle.ad_mul(A, B, 65535))
        ok &= np.array_equal(sr.to_host(dAc).astype(np.int64), oracle.ad_closure(A, 65535))
        out["parity"] = {"all_four_outputs": True, "bit_exact": bool(ok)}
    return out


def run_boolmul(args, torch, sr, synthgen):
    """Boolean product A * A of the D = 16384 Boolean input (bit-packed): the
    default path (value), with the bit-sliced, four-Russians and matrix-core
    (4-bit float and int8 operands) paths reported beside it; every path's
    product equal, the default's against the oracle's whole product."""
    import numpy as np
    import oracle
    D = 16384
    W = synthgen.cfg_bool16384(D=D)
    A = sr.to_device(sr.SR_BOOL, W, cols=D)
    C1 = sr.empty(sr.SR_BOOL, D, D)
    C2 = sr.empty(sr.SR_BOOL, D, D)
    C3 = sr.empty(sr.SR_BOOL, D, D)
    C4 = sr.empty(sr.SR_BOOL, D, D)
    fb = lambda i: sr.semiring_mul(sr.SR_BOOL, C1, A, A, K=D, N=D)
    fm = lambda i: sr.semiring_mul(sr.SR_BOOL, C2, A, A, K=D, N=D, flags=sr.SR_BOOL_MFMA)
    fw = lambda i: sr.semiring_mul(sr.SR_BOOL, C3, A, A, K=D, N=D, flags=sr.SR_BOOL_BITWISE)
    fr = lambda i: sr.semiring_mul(sr.SR_BOOL, C4, A, A, K=D, N=D, flags=sr.SR_BOOL_M4R)
    for _ in range(max(1, args.warmup)):
        fb(0)
        fm(0)
        fw(0)
        fr(0)
    tb = timed(torch, fb, args.steps)
    tm = timed(torch, fm, args.steps)
    tw = timed(torch, fw, args.steps)
    tr = timed(torch, fr, args.steps)
    os.environ["SR_MFMA_FORMAT"] = "i8"
    C5 = sr.empty(sr.SR_BOOL, D, D)
    fi = lambda i: sr.semiring_mul(sr.SR_BOOL, C5, A, A, K=D, N=D, flags=sr.SR_BOOL_MFMA)
    fi(0)
    ti = timed(torch, fi, args.steps)
    os.environ.pop("SR_MFMA_FORMAT", None)
    out = {"metric": "semiring updates/s (R*K*N/t) Boolean product 16384^3",
           "value": float(D) ** 3 / (tb * 1e-3), "unit": "updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": tb,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bits",
           "data": "synthetic",
           "config": {"workload": "bool_product_D16384", "D": D, "parallelism": "single_gpu"},
           "nominal_updates_vs_bitwise_roofline": float(D) ** 3 / (tb * 1e-3) / PEAK_BOOL,
           "bitwise_path": {"ms_per_step": tw, "value": float(D) ** 3 / (tw * 1e-3),
                            "fraction_of_bitwise_roofline": float(D) ** 3 / (tw * 1e-3) / PEAK_BOOL},
           "m4r_path": {"ms_per_step": tr, "value": float(D) ** 3 / (tr * 1e-3)},
           # the matrix-core path: one MAC per nominal update; 4-bit float
           # operands (MI355X dense fp4: 10.1 PFLOP/s = 5.05e15 MAC/s) and
           # int8 ones (5.0 POP/s = 2.5e15 MAC/s)
           "mfma_path": {"ms_per_step": tm, "value": float(D) ** 3 / (tm * 1e-3),
                         "operands": "fp4 e2m1",
                         "fraction_of_fp4_mfma_peak": float(D) ** 3 / (tm * 1e-3) / PEAK_F4_MAC,
                         "speedup_vs_default": tb / tm},
           "mfma_int8_path": {"ms_per_step": ti, "value": float(D) ** 3 / (ti * 1e-3),
                              "fraction_of_int8_mfma_peak": float(D) ** 3 / (ti * 1e-3) / PEAK_I8_MAC,
                              "speedup_vs_default": tb / ti}}
    torch.cuda.synchronize()
    out["paths_equal"] = bool(torch.equal(C1, C2) and torch.equal(C1, C3) and torch.equal(C1, C4)
                              and torch.equal(C1, C5))
    if not args.no_cpu_baseline or not args.no_parity:
        # the oracle's bit-packed product on all host threads: the CPU
        # baseline, and every word of the parity check
        oracle.set_threads(args.cpu_threads)
        t0 = time.perf_counter()
        want = oracle.bool_mul_words(W, W, D, D)
        dt = time.perf_counter() - t0
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = {"value": float(D) ** 3 / dt, "unit": "updates/s",
                                   "cores": args.cpu_threads, "kind": "oracle",
                                   "sample": "the whole 16384^3 product (nominal updates; the "
                                             "bit-packed loop skips rows whose bit is clear)",
                                   "cpu": host_cpu()}
        if not args.no_parity:
            nw = D // 64
            out["parity"] = {"words_compared": int(D * nw), "whole_matrix": True,
                             "bit_exact": bool(np.array_equal(sr.to_host(C1)[:, :nw],
                                                              want[:, :nw]))}
    return out


def run_add(args, torch, sr, synthgen):
    """Entrywise (+) of two 8192 x 8192 uint16 matrices (reads 256 MiB,
    writes 128 MiB): the HBM-bound step, and the streaming kernel of known
    size that calibrates the FETCH_SIZE / WRITE_SIZE counters.  The whole
    result is compared with the oracle's entrywise maximum."""
    import numpy as np
    D = 8192
    kind = sr.SR_ANTIDIST_U16
    hA = synthgen.cfg_antidist(D=D, which=0)
    hB = synthgen.cfg_antidist(D=D, which=1)
    A = sr.to_device(kind, hA)
    B = sr.to_device(kind, hB)
    C = sr.empty(kind, D, D)
    f = lambda i: sr.semiring_add(kind, C, A, B)
    for _ in range(args.warmup):
        f(0)
    steps = max(args.steps, 20)
    ms = timed(torch, f, steps)
    nbytes = 3 * D * D * 2
    gbs = nbytes / (ms * 1e-3) / 1e9
    out = {"metric": "HBM GB/s of semiring_add (entrywise max) 8192x8192 uint16",
           "value": gbs, "unit": "GB/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u16", "data": "synthetic",
           "config": {"workload": "antidist_u16_add_8192", "bytes_per_call": nbytes,
                      "parallelism": "single_gpu"},
           "roofline": {"bound": "hbm", "kernel": "k_ewise<2, EW_OR, NT=true>", "achieved": gbs, "peak": 8000.0,
                        "unit": "GB/s", "frac": gbs / 8000.0, "traffic": None}}
    if not args.no_cpu_baseline or not args.no_parity:
        import oracle
        t0 = time.perf_counter()
        want = oracle.ewise("or", hA, hB)
        dt = time.perf_counter() - t0
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = {"value": nbytes / dt / 1e9, "unit": "GB/s", "cores": 1,
                                   "kind": "oracle",
                                   "sample": "the whole 8192 x 8192 call (numpy, one thread)",
                                   "cpu": host_cpu()}
        if not args.no_parity:
            got = sr.to_host(C)[:, :D].astype(np.int64)
            out["parity"] = {"entries_compared": D * D, "whole_matrix": True,
                             "bit_exact": bool(np.array_equal(got, want))}
    return out


def run_serve(args, torch, sr, synthgen):
    """Serving: closure requests of log-uniform size in [64, 8192], half
    Boolean (p = 0.02) and half uint16 anti-distance (configuration-2
    generator), Poisson arrivals at 80% of the serial service rate of the same
    trace; served (continuous batching, footprint admission, concurrent
    slots) against the same trace solved one at a time.  Every served result
    is compared with the oracle: whole closures up to 2048 vertices, sampled
    rows (per-source shortest paths / breadth-first search) above."""
    import numpy as np
    from paper_1705_08743_amd.serve import ClosureServer, Request
    kinds = {"bool": sr.SR_BOOL, "u16": sr.SR_ANTIDIST_U16}

    def make(trace):
        return [(kinds[k], n, synthgen.serving_request(n, k, seed)) for n, k, seed in trace]

    log("generating %d requests ..." % args.serve_requests)
    reqs = make(synthgen.serving_trace(args.serve_requests))
    server = ClosureServer(budget_bytes=int(args.serve_budget_gb * (1 << 30)), slots=4)
    fresh = lambda items, arr: [Request(i, k, n, h, a) for i, ((k, n, h), a) in
                                enumerate(zip(items, arr))]
    zeros = np.zeros(len(reqs))
    # warm-up (allocator, code objects, pinned copies), then the trace's own
    # serial service time: its serial makespan with every request waiting
    log("warm-up and serial service time ...")
    server.run(fresh(reqs, zeros), "served")
    sat_serial = server.run(fresh(reqs, zeros), "serial")
    mean_service = sat_serial["makespan_s"] / len(reqs)
    rate = 0.8 / mean_service
    arrivals = synthgen.poisson_arrivals(len(reqs), rate, synthgen.generator(synthgen.config_seed(5) + 7))
    log("replaying at %.1f requests/s ..." % rate)
    served_reqs = fresh(reqs, arrivals)
    served = server.run(served_reqs, "served")
    serial_reqs = fresh(reqs, arrivals)
    serial = server.run(serial_reqs, "serial")
    same = all(np.array_equal(a.result, b.result) for a, b in zip(served_reqs, serial_reqs))
    del serial_reqs
    sat_served = server.run(fresh(reqs, zeros), "served")
    span = float(arrivals[-1] - arrivals[0])
    out = {"metric": "served requests/s (closure requests, Poisson at 80% of serial capacity); "
                     "p50/p99 latency vs serial",
           "value": served["throughput_rps"], "unit": "requests/s", "n_gpus": 1,
           "steps": len(reqs), "warmup": 1, "ms_per_step": 1e3 / served["throughput_rps"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "u16+bits", "data": "synthetic",
           "config": {"workload": "serving_mixed_closures", "requests": len(reqs),
                      "n": "log-uniform [64,8192]", "mix": "50% Boolean p=0.02, 50% uint16 p=0.05",
                      "arrival_rate_rps": rate, "mean_serial_service_ms": mean_service * 1e3,
                      "offered_load": rate * mean_service,
                      "realized_load": sat_serial["makespan_s"] / span if span > 0 else None,
                      "budget_gb": args.serve_budget_gb, "slots": 4, "batch_n": 256,
                      "parallelism": "single_gpu"},
           "served": served, "serial": serial,
           "saturated": {"served_rps": sat_served["throughput_rps"],
                         "serial_rps": sat_serial["throughput_rps"],
                         "served_updates_per_s": sat_served["updates_per_s"],
                         "serial_updates_per_s": sat_serial["updates_per_s"],
                         "throughput_speedup": sat_served["throughput_rps"] / sat_serial["throughput_rps"],
                         "batched_requests": sat_served["batched_requests"]},
           "p99_speedup_vs_serial": serial["p99_ms"] / served["p99_ms"],
           "p50_speedup_vs_serial": serial["p50_ms"] / served["p50_ms"],
           "parity": {"served_equals_serial_all_requests": bool(same)}}
    if not args.no_parity:
        log("oracle check of every served result ...")
        out["parity"].update(serve_oracle_parity(sr, served_reqs, args.cpu_threads))
    return out


def serve_oracle_parity(sr, reqs, threads, whole_max=2048, rows_per_request=4):
    """Every served result against the oracle: the whole closure (Warshall's
    loop) for requests of at most whole_max vertices, and for larger ones
    sampled rows from the oracle's per-source path definition (Dijkstra on
    distances, breadth-first search for Boolean), rows 0, n - 1 and two
    seeded ones."""
    import numpy as np
    import oracle
    import synthgen
    oracle.set_threads(threads)
    gen = synthgen.generator(synthgen.config_seed(5) + 11)
    whole = rows = entries = 0
    bad = []
    for r in reqs:
        n = r.n
        if r.kind == sr.SR_BOOL:
            got = r.result.view(np.uint64)
            nw = (n + 63) // 64
            if n <= whole_max:
                ok = np.array_equal(got, oracle.bool_closure_words(r.host, n)[:, :nw])
                whole += 1
                entries += n * n
            else:
                sel = sorted({0, n - 1, *gen.integers(0, n, size=rows_per_request - 2).tolist()})
                want = oracle.bool_closure_rows_words(r.host, n, np.array(sel))
                ok = np.array_equal(got[sel], want[:, :nw])
                rows += len(sel)
                entries += len(sel) * n
        else:
            A = r.host[:, :n]
            if n <= whole_max:
                ok = np.array_equal(r.result.astype(np.int64), oracle.ad_closure(A, 65535))
                whole += 1
                entries += n * n
            else:
                sel = sorted({0, n - 1, *gen.integers(0, n, size=rows_per_request - 2).tolist()})
                want = oracle.ad_closure_rows(A, 65535, np.array(sel))
                ok = np.array_equal(r.result[sel].astype(np.int64), want)
                rows += len(sel)
                entries += len(sel) * n
        if not ok:
            bad.append(r.rid)
    return {"oracle_requests_checked": len(reqs), "oracle_whole_closures": whole,
            "oracle_sampled_rows": rows, "oracle_entries_compared": int(entries),
            "oracle_bit_exact": not bad, "oracle_mismatches": bad[:10]}


TILE_NAMES = {1: "64x16", 2: "64x32", 3: "64x64"}


def prepared_graph(torch, sr, kind, arena):
    """The batch prepared once (plan built and uploaded, update tiles
    autotuned) and its whole closure captured into one graph."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        pb = sr.PreparedBatch(kind, arena)
        tile = pb.autotune()
        pb.run()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        pb.run()
    torch.cuda.synchronize()
    return pb, g, tile


def run_batched(args, torch, sr, synthgen):
    """4096 graphs, log-uniform sizes in [32, 1024], uint16 (then uint8,
    Boolean and uint32): the prepared batch replayed as one graph launch,
    against one closure_batched call and against one closure() call per graph
    on the same stream."""
    import numpy as np
    import oracle
    log("generating 4096 graphs ...")
    batch = synthgen.cfg_batch()
    mats = [synthgen.encode_antidist(n, r, c, w, np.uint16) for n, r, c, w in batch]
    kind = sr.SR_ANTIDIST_U16
    sizes = [m.shape[0] for m in mats]
    # the batch lives in one device arena (its pointer arrays built once)
    src = sr.BatchArena(kind, sizes)
    src.load(mats)
    work = sr.BatchArena(kind, sizes, zero=False)
    views = [work.view(i) for i in range(len(mats))]
    upd = float(sum(float(n) ** 3 for n in sizes))

    def reset():
        work.copy_(src)

    log("preparing, autotuning and capturing the batch ...")
    reset()
    pb, g, tile = prepared_graph(torch, sr, kind, work)
    for _ in range(max(1, args.warmup)):
        reset()
        g.replay()
        reset()
        sr.closure_batched(kind, work)
    times_g, times_b, times_s = [], [], []
    for _ in range(max(1, args.steps // 2)):
        reset()
        times_g.append(timed(torch, lambda i: g.replay(), 1))
        reset()
        times_b.append(timed(torch, lambda i: sr.closure_batched(kind, work), 1))
        reset()
        times_s.append(timed(torch, lambda i: [sr.closure(kind, t) for t in views], 1))
    tg, tb, ts = min(times_g), min(times_b), min(times_s)
    out = {"metric": "semiring updates/s (sum n³/t) batched closure, 4096 graphs",
           "value": upd / (tg * 1e-3), "unit": "updates/s", "n_gpus": 1,
           "steps": len(times_g), "warmup": args.warmup, "ms_per_step": tg,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u16",
           "data": "synthetic",
           "config": {"workload": "batched_antidist_u16_4096", "graphs": len(mats),
                      "n": "log-uniform [32,1024]", "edge_p": "U[0.01,0.2]",
                      "distances": "U[1,200]", "parallelism": "single_gpu",
                      "launch": "one graph replay of the prepared batch",
                      "update_tile": TILE_NAMES.get(tile, str(tile))},
           "closure_batched_ms": tb, "serial_ms": ts, "speedup_vs_serial": ts / tg,
           "total_updates": upd,
           "fraction_of_valu_roofline": upd / (tg * 1e-3) / PEAK_ANTIDIST}
    if not args.no_parity or not args.no_cpu_baseline:
        reset()
        g.replay()
        ref = sr.BatchArena(kind, sizes, zero=False)
        ref.copy_(src)
        sr.closure_batched(kind, ref)
        torch.cuda.synchronize()
        same = bool(torch.equal(ref.buf, work.buf))
        del ref
        log("the oracle on all %d graphs ..." % len(mats))
        oracle.set_threads(args.cpu_threads)
        bad, dt = oracle_batch_parity(arena_mats(work, np.uint16), mats,
                                      lambda m: oracle.ad_closure(m, 65535))
        if not args.no_parity:
            out["parity"] = {"graphs_compared": len(mats), "graphs_differing": bad,
                             "bit_exact": bad == 0, "graph_replay_equals_closure_batched": same}
        if not args.no_cpu_baseline:
            # one thread on every 16th graph (a bounded sample of the batch)
            oracle.set_threads(1)
            sample = mats[::16]
            t1 = time.perf_counter()
            for m in sample:
                oracle.ad_closure(m, 65535)
            dt1 = time.perf_counter() - t1
            oracle.set_threads(args.cpu_threads)
            upd1 = float(sum(float(m.shape[0]) ** 3 for m in sample))
            out["cpu_baseline"] = {"value": upd / dt, "unit": "updates/s",
                                   "cores": args.cpu_threads, "kind": "oracle",
                                   "sample": "the whole batch, one oracle closure per graph "
                                             "(%.3g updates, %.1f s)" % (upd, dt),
                                   "seconds": dt, "cpu": host_cpu(),
                                   "one_thread": {"value": upd1 / dt1, "unit": "updates/s",
                                                  "sample": "every 16th graph on 1 thread "
                                                            "(%.3g updates, %.1f s)" % (upd1, dt1)}}
    del g
    pb.close()
    # the same 4096 topologies and distances as uint8 (binary16 working form)
    mats8 = [synthgen.encode_antidist(n, r, c, w, np.uint8) for n, r, c, w in batch]
    del work, views
    src8 = sr.BatchArena(sr.SR_ANTIDIST_U8, sizes)
    src8.load(mats8)
    work8 = sr.BatchArena(sr.SR_ANTIDIST_U8, sizes, zero=False)
    work8.copy_(src8)
    pb8, g8, tile8 = prepared_graph(torch, sr, sr.SR_ANTIDIST_U8, work8)
    for _ in range(max(1, args.warmup)):
        work8.copy_(src8)
        g8.replay()
    times8, times8b = [], []
    for _ in range(max(1, args.steps // 2)):
        work8.copy_(src8)
        times8.append(timed(torch, lambda i: g8.replay(), 1))
        work8.copy_(src8)
        times8b.append(timed(torch, lambda i: sr.closure_batched(sr.SR_ANTIDIST_U8, work8), 1))
    t8, t8b = min(times8), min(times8b)
    out["uint8"] = {"ms": t8, "value": upd / (t8 * 1e-3), "closure_batched_ms": t8b,
                    "update_tile": TILE_NAMES.get(tile8, str(tile8)),
                    "fraction_of_valu_roofline_u8": upd / (t8 * 1e-3) / PEAK_ANTIDIST_U8}
    if not args.no_parity:
        work8.copy_(src8)
        g8.replay()
        torch.cuda.synchronize()
        bad8, _ = oracle_batch_parity(arena_mats(work8, np.uint8), mats8,
                                      lambda m: oracle.ad_closure(m, 255))
        out["uint8"]["parity"] = {"graphs_compared": len(mats8), "graphs_differing": bad8,
                                  "bit_exact": bad8 == 0}
    del g8
    pb8.close()
    del work8, src8
    # the same topologies as Boolean graphs (bit-packed, closed as {0, 255}
    # anti-distance matrices) and with 32-bit entries, each as one graph launch
    for name, kind in (("boolean", sr.SR_BOOL), ("uint32", sr.SR_ANTIDIST_U32)):
        if kind == sr.SR_BOOL:
            hm = []
            for n, r, c, w in batch:
                d = np.zeros((n, n), np.uint8)
                d[r, c] = 1
                hm.append(synthgen.pack_bits(d, synthgen.aligned_ld_words(max(n, 1))))
        else:
            hm = [synthgen.encode_antidist(n, r, c, w, np.uint32) for n, r, c, w in batch]
        srcx = sr.BatchArena(kind, sizes)
        srcx.load(hm)
        workx = sr.BatchArena(kind, sizes, zero=False)
        workx.copy_(srcx)
        pbx, gx, tilex = prepared_graph(torch, sr, kind, workx)
        tx = []
        for _ in range(max(1, args.steps // 2)):
            workx.copy_(srcx)
            tx.append(timed(torch, lambda i: gx.replay(), 1))
        out[name] = {"ms": min(tx), "value": upd / (min(tx) * 1e-3),
                     "update_tile": TILE_NAMES.get(tilex, str(tilex))}
        if kind == sr.SR_ANTIDIST_U32:
            out[name]["fraction_of_valu_roofline_u32"] = upd / (min(tx) * 1e-3) / PEAK_ANTIDIST32
        if not args.no_parity:
            workx.copy_(srcx)
            gx.replay()
            torch.cuda.synchronize()
            if kind == sr.SR_BOOL:
                bad, _ = oracle_batch_parity(
                    arena_mats(workx, np.uint64), hm,
                    lambda m: oracle.bool_closure_words(m, m.shape[0])[:, :-(-m.shape[0] // 64)])
            else:
                bad, _ = oracle_batch_parity(arena_mats(workx, np.uint32), hm,
                                             lambda m: oracle.ad_closure(m, 2 ** 32 - 1))
            out[name]["parity"] = {"graphs_compared": len(hm), "graphs_differing": bad,
                                   "bit_exact": bad == 0}
        del gx
        pbx.close()
        del workx, srcx
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="fw8192",
                    choices=["fw8192", "u8fw8192", "dfw8192", "u32fw8192", "bool16384",
                             "boolmul16384", "mul1024", "small", "batched", "add8192", "serve"])
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-budget-gb", type=float, default=16.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--cpu1-seconds", type=float, default=5.0,
                    help="bound of the one-thread oracle sample")
    ap.add_argument("--cpu-threads", type=int, default=oracle_threads())
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see the sharding design notes); got --gpus %d" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    import paper_1705_08743_amd as sr
    import synthgen
    sr.lib()  # fails loudly when the library is not built

    metric = "semiring updates/s (D³/t) anti-distance FW D=8192; served p50/p99 vs serial"
    if args.workload == "fw8192":
        out = run_fw(args, torch, sr, sr.SR_ANTIDIST_U16, 8192,
                     lambda: synthgen.cfg_antidist(D=8192), "fw8192", 65535, metric)
        out["config"] = {"workload": "antidist_u16_floyd_warshall_D8192", "D": 8192,
                         "entries": "uint16, S=65535", "edge_p": 0.05,
                         "distances": "U[1,1000]; 1% U[64536,65534]",
                         "seed": synthgen.config_seed(2), "pivot_block": 128,
                         "parallelism": "single_gpu"}
    elif args.workload == "u8fw8192":
        out = run_fw(args, torch, sr, sr.SR_ANTIDIST_U8, 8192,
                     lambda: synthgen.cfg_antidist_u8(D=8192), "u8fw8192", 255,
                     "semiring updates/s (D³/t) anti-distance FW D=8192 uint8",
                     peak=PEAK_ANTIDIST_U8)
        out["config"] = {"workload": "antidist_u8_floyd_warshall_D8192", "D": 8192,
                         "entries": "uint8, S=255", "edge_p": 0.05, "distances": "U[1,200]",
                         "pivot_block": 128, "parallelism": "single_gpu"}
    elif args.workload == "dfw8192":
        def dist_input():
            import numpy as np
            A = synthgen.cfg_antidist(D=8192)[:, :8192]
            return (65535 - A.astype(np.int64)).astype(np.uint16)
        out = run_fw(args, torch, sr, sr.SR_DISTANCE_U16, 8192, dist_input, "dfw8192", 65535,
                     "semiring updates/s (D³/t) distance-matrix closure (min, saturating +) D=8192",
                     dual=True)
        out["config"] = {"workload": "distance_u16_closure_D8192", "D": 8192,
                         "entries": "uint16 distances, 65535 = no path", "edge_p": 0.05,
                         "distances": "U[1,1000]; 1% U[64536,65534]", "pivot_block": 128,
                         "parallelism": "single_gpu"}
    elif args.workload == "u32fw8192":
        def u32_input():
            import numpy as np
            A = synthgen.cfg_antidist(D=8192)[:, :8192].astype(np.int64)
            # the same distances, encoded with S = 2^32 - 1 (heavy edges no
            # longer saturate after one more hop)
            return np.where(A > 0, (2 ** 32 - 1) - (65535 - A), 0).astype(np.uint32)
        out = run_fw(args, torch, sr, sr.SR_ANTIDIST_U32, 8192, u32_input, "u32fw8192",
                     2 ** 32 - 1, "semiring updates/s (D³/t) anti-distance FW D=8192 uint32",
                     peak=PEAK_ANTIDIST32, kernel="k_ad32_update (update phase)")
        out["config"] = {"workload": "antidist_u32_floyd_warshall_D8192", "D": 8192,
                         "entries": "uint32, S=2^32-1", "edge_p": 0.05,
                         "distances": "U[1,1000]; 1% U[64536,65534]", "pivot_block": 128,
                         "parallelism": "single_gpu"}
    elif args.workload == "bool16384":
        out = run_bool(args, torch, sr, synthgen)
    elif args.workload == "boolmul16384":
        out = run_boolmul(args, torch, sr, synthgen)
    elif args.workload == "mul1024":
        out = run_mul(args, torch, sr, synthgen)
    elif args.workload == "small":
        out = run_small(args, torch, sr, synthgen)
    elif args.workload == "add8192":
        out = run_add(args, torch, sr, synthgen)
    elif args.workload == "serve":
        out = run_serve(args, torch, sr, synthgen)
    else:
        out = run_batched(args, torch, sr, synthgen)
    out["library"] = sr.version()
    out["device"] = torch.cuda.get_device_name(0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
