"""Benchmark of the wavelet-tree hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload text_zipf|large_alpha|forest|serve|bitvec]
                    [--l2-bits B] [--sample-rate S] [--no-learned] [--no-cpu-baseline]

One step = one pass of the whole hot path over one batch of synthetic input already resident in
HBM: build the level-wise wavelet tree of n symbols (histogram, node tables, every level's bits,
rank directory, select samples and partition), train its learned select index, answer q access,
q rank, q select and q learned-select queries, then free the tree. Default workload: n = 2^30 u8 symbols, alphabet 256, Zipf(1.0) frequencies over
a seeded permutation, q = 2^26 queries of each kind.

Prints one JSON line. `value` is (symbols built + queries answered) per second over the timed
steps; the per-part rates are in `rates`. `roofline` covers the kernel with the most time in a
step; `roofline_build` the build's level pass, timed with HIP events recorded by the library
around every level launch on the build stream; `roofline_build_total` the whole build (histogram
read plus every level pass, over the median build time).
`cpu_baseline` times the plain CPU oracle on a bounded prefix of the same workload.
`rates.select_unbinned` compares plain and learned select on 2^24 of the queries asked in batches of
2^15 (below the binning size), outside the timed steps.

--workload forest: 1024 u16 sequences (lengths log-uniform in [2^10, 2^24], alphabets log-uniform in
[4, 2^16], Zipf 1.0) built as one forest (one captured graph launch, |L2| and s from the autotuner)
plus 2^24 mixed access/rank/select queries across the trees; also timed the plain way (one wt_build
and three query calls per tree) for the comparison.
--workload serve: 64 resident trees of 2^26 u8 Zipf(1.0) symbols; query batches of log-uniform size
in [1, 2^20] (70 % select, 20 % rank, 10 % access) from page-locked host memory, replayed at
saturation and at Poisson arrivals of 0.5, 0.8 and 0.95 of the saturation rate; p50/p99 latency and
queries/s. (Selects inside mixed batches use the plain sampled search.)

The default run also measures, outside its timed steps, the wavelet matrix and the Huffman-shaped tree
of the same sequence answering the same queries (keys `matrix`, `huffman`), queries from host memory
(wt_query_host, 10^5..10^7 of each kind, page-locked and pageable arrays; key `host_queries`), the
chunked build from host memory against copy-then-build (wt_build_host, 2^27-symbol chunks; key
`host_build`), the
large-alphabet configuration (2^28 u32 symbols, sigma 2^20; key `large_alpha`), the batched forest
build and its mixed queries (three builds of the forest workload below, without the one-tree-at-a-time
comparison; key `forest`) and the rank/select
benchmark of plain bit arrays (2^32 bits, fill 10/50/90 %, uniform and adversarial placement, |L2| 512,
s 16384, 10^8 queries of each of rank0/rank1/select0/select1; key `bitvec`).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
PMC_FILE = os.path.join(ROOT, "profiles", "level_kernel_text_zipf_pmc.json")
LEVEL_SRCS = [os.path.join(ROOT, "paper_2505_03372_amd", "csrc", f) for f in ("wt_build_dev.h", "wt_build.hip")]
QUERY_PMC_FILE = os.path.join(ROOT, "profiles", "query_kernels_text_zipf_pmc.json")
QUERY_SRCS = [os.path.join(ROOT, "paper_2505_03372_amd", "csrc", f)
              for f in ("wt_query_dev.h", "wt_query.hip", "wt_learn_dev.h", "wt_learn.hip", "wt_internal.h")]


def level_launch_bytes(info: dict, w: int) -> list:
    """Algorithmic HBM bytes of each level-kernel launch: read the level (w B/symbol), write the
    next level's sequence (w B/symbol, not at the last level), write the bits (1/8 B/symbol), the L1
    and L2 entries and the select samples."""
    L = info["levels"]
    s = info["sample_rate"]
    out = []
    for l in range(L):
        nl = info["level_n"][l]
        ones = info["level_ones"][l]
        b = nl * w                                      # read level l
        if l + 1 < L:
            b += info["level_n"][l + 1] * w             # write level l + 1
        b += (nl + 63) // 64 * 8                        # bit words
        b += ((nl + 65535) // 65536) * 8                # L1
        b += ((nl + info["l2_bits"] - 1) // info["l2_bits"]) * 2  # L2
        b += (ones // s + (nl - ones) // s) * 8         # samples
        out.append(b)
    return out


def source_hash(paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(per_launch_alg: float):
    """HBM traffic of the level kernel from the committed rocprofv3 counter summary (taken on the
    2^30 u8 Zipf workload), if it was taken on the current kernel source."""
    if not os.path.exists(PMC_FILE):
        return None
    with open(PMC_FILE) as f:
        pmc = json.load(f)
    if pmc.get("source_sha256_16") != source_hash(LEVEL_SRCS):
        return None
    return pmc.get("traffic_bytes_per_launch")


def load_query_traffic(kernel: str, q: int):
    """HBM traffic of a query kernel launch from the committed counter summary (same sources, same q)."""
    if not os.path.exists(QUERY_PMC_FILE):
        return None
    with open(QUERY_PMC_FILE) as f:
        pmc = json.load(f)
    if pmc.get("source_sha256_16") != source_hash(QUERY_SRCS) or pmc.get("queries_per_launch") != q:
        return None
    k = pmc.get("kernels", {}).get(kernel)
    return k["traffic_bytes"] if k else None


def _short_kernel(name: str) -> str:
    """'void wt::k_select<9, 1024u, 0>(...)' -> 'k_select<9, 1024u>' (the shape argument 0, the tree,
    dropped: the names the bench line uses); other shapes and kernels keep their arguments."""
    k = name.split("(")[0].replace("void ", "").replace("wt::", "").strip()
    return k[:-4] + ">" if k.endswith(", 0>") else k


def profile_summary(d: str) -> None:
    """Writes the summaries under profiles/ from the rocprofv3 runs of PROFILE_COMMANDS kept in `d`
    (trace/, fetch/, write/, l2/ with their CSV files, and the bench JSON lines trace.json and
    fetch.json): the kernel statistics of the default text_zipf run against the bench line of the same
    run, and the HBM traffic and L2 hit rate of the level kernel and the binned query kernels. The
    counters are read per dispatch (FETCH_SIZE and WRITE_SIZE in KiB) and scaled by what they read for
    the run's 1 GiB device copy."""
    import csv

    def rows(sub, name):
        with open(os.path.join(d, sub, name)) as f:
            return list(csv.DictReader(f))

    def bench_line(name):
        with open(os.path.join(d, name)) as f:
            return json.loads(f.read().strip().splitlines()[-1])

    out_dir = os.path.join(ROOT, "profiles")
    cmd = PROFILE_COMMANDS
    # kernel statistics
    stats = rows("trace", "run_kernel_stats.csv")
    tl = bench_line("trace.json")
    tot = sum(float(r["TotalDurationNs"]) for r in stats)
    lines = ["# all kernels of the default bench, text_zipf (2^30 u8, 2^26 queries per kind): rocprofv3 kernel trace",
             "", "Command (repository root on the GPU box, `TMPDIR=/tmp`):", "", "    " + cmd["trace"], "",
             "Kernel statistics (`run_kernel_stats.csv`, top entries):", "",
             "| kernel | calls | avg µs | total ms | % |", "|---|---|---|---|---|"]
    by = {}
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:16]:
        k = _short_kernel(r["Name"])
        by[k] = r
        lines.append("| %s | %s | %.1f | %.1f | %.2f |" % (k, r["Calls"], float(r["AverageNs"]) / 1e3,
                                                        float(r["TotalDurationNs"]) / 1e6,
                                                        100.0 * float(r["TotalDurationNs"]) / tot))
    for key, what in (("roofline", "Kernel with the most time per step"), ("roofline_build", "Build kernel")):
        rf = tl[key]
        match = [r for r in stats if _short_kernel(r["Name"]).replace("uint8_t", "unsigned char")
                 .startswith(rf["kernel"].replace("uint8_t", "unsigned char").rstrip(">"))]
        if match:
            r = match[0]
            lines += ["", "%s `%s`: rocprofv3 average %.1f µs over %s launches; the bench line of the same run "
                      "(`%s`) reports avg_launch_ms = %.4f (HIP events around each launch), achieved %.0f GB/s = "
                      "%.3f of %.0f GB/s." % (what, _short_kernel(r["Name"]), float(r["AverageNs"]) / 1e3, r["Calls"],
                                               key, rf["avg_launch_ms"], rf["achieved"], rf["frac"], rf["peak"])]
    with open(os.path.join(out_dir, "kernels_text_zipf_trace.md"), "w") as f:
        f.write("\n".join(lines) + "\n")

    # counters
    fl = bench_line("fetch.json")
    fetch, write, l2 = rows("fetch", "run_counter_collection.csv"), rows("write", "run_counter_collection.csv"), \
        rows("l2", "run_counter_collection.csv")

    def vals(rs, counter, pred):
        return [float(r["Counter_Value"]) for r in rs if r["Counter_Name"] == counter and pred(r["Kernel_Name"])]

    def copy_scale(rs, counter):
        v = vals(rs, counter, lambda k: "copyBuffer" in k)
        return float(fl["calibration_copy_bytes"]) / (max(v) * 1024.0)

    fs, ws = copy_scale(fetch, "FETCH_SIZE"), copy_scale(write, "WRITE_SIZE")

    def traffic(pred):
        fv, wv = vals(fetch, "FETCH_SIZE", pred), vals(write, "WRITE_SIZE", pred)
        h, m = sum(vals(l2, "TCC_HIT_sum", pred)), sum(vals(l2, "TCC_MISS_sum", pred))
        return (len(fv), float(np.mean(fv)) * 1024 * fs, float(np.mean(wv)) * 1024 * ws,
                h / (h + m) if h + m else None)

    lvl = lambda k: _short_kernel(k).startswith("k_level<unsigned char, false")
    n_l, f_l, w_l, hit_l = traffic(lvl)
    alg_l = fl["roofline_build"]["bytes_per_launch"]
    lj = {"kernel": "k_level<unsigned char, false>", "workload": "level_kernel_text_zipf",
          "source_sha256_16": source_hash(LEVEL_SRCS), "launches": n_l, "fetch_scale": fs, "write_scale": ws,
          "fetch_bytes_per_launch": f_l, "write_bytes_per_launch": w_l, "traffic_bytes_per_launch": f_l + w_l,
          "algorithmic_bytes_per_launch": alg_l, "l2_hit_rate": hit_l, "commands": [cmd["fetch"], cmd["write"], cmd["l2"]]}
    with open(os.path.join(out_dir, "level_kernel_text_zipf_pmc.json"), "w") as f:
        json.dump(lj, f, indent=1)
    q = fl["config"]["queries_per_kind"]
    qj = {"source_sha256_16": source_hash(QUERY_SRCS), "queries_per_launch": q, "kernels": {},
          "commands": [cmd["fetch"], cmd["write"], cmd["l2"]]}
    for name in ("k_access<9, 1024u>", "k_rank<9, 1024u>", "k_select<9, 1024u>", "k_select_learned<9, 1024u>"):
        nk, fq, wq, hq = traffic(lambda k, name=name: _short_kernel(k) == name)
        alg = 64.0 * (int(fl["config"]["sigma"]) - 1).bit_length() * q  # levels of the tree: ceil(lg sigma)
        qj["kernels"][name] = {"launches": nk, "fetch_bytes": fq, "write_bytes": wq, "traffic_bytes": fq + wq,
                               "algorithmic_bytes": alg, "l2_hit_rate": hq}
    with open(os.path.join(out_dir, "query_kernels_text_zipf_pmc.json"), "w") as f:
        json.dump(qj, f, indent=1)
    md = ["# level and query kernels, text_zipf (2^30 u8, 2^26 queries per kind): HBM traffic and L2 hits", "",
          "Commands (repository root on the GPU box, `TMPDIR=/tmp`; one counter set per run):", ""]
    md += ["    " + cmd[k] for k in ("fetch", "write", "l2")]
    md += ["", "FETCH_SIZE and WRITE_SIZE are KiB per dispatch; scaled by what they read for the run's 1 GiB device "
           "copy (FETCH x %.3f, WRITE x %.3f). Algorithmic bytes: the level pass's stream (bench.py "
           "`level_launch_bytes`); a query kernel's 64 B (one L2 block of bits) per level per query." % (fs, ws), "",
           "| kernel | launches | FETCH (GB) | WRITE (GB) | traffic / algorithmic | L2 hit rate |",
           "|---|---|---|---|---|---|",
           "| k_level<unsigned char, false> (per launch) | %d | %.3f | %.3f | %.3f | %.3f |"
           % (n_l, f_l / 1e9, w_l / 1e9, (f_l + w_l) / alg_l, hit_l or 0.0)]
    for name, k in qj["kernels"].items():
        md.append("| %s | %d | %.3f | %.3f | %.2f | %.3f |" % (name, k["launches"], k["fetch_bytes"] / 1e9,
                                                             k["write_bytes"] / 1e9,
                                                             k["traffic_bytes"] / k["algorithmic_bytes"],
                                                             k["l2_hit_rate"] or 0.0))
    md += ["", "Source hashes (sha256/16): level kernel %s, query kernels %s." % (lj["source_sha256_16"],
                                                                               qj["source_sha256_16"])]
    with open(os.path.join(out_dir, "kernel_traffic_text_zipf_pmc.md"), "w") as f:
        f.write("\n".join(md) + "\n")
    if os.path.isdir(os.path.join(d, "forest")):
        forest_summary(d, out_dir)
    print("profiles written from", d)


def forest_summary(d: str, out_dir: str) -> None:
    """profiles/forest_build_graph_trace.md from the kernel trace of PROFILE_COMMANDS["forest"]: kernel
    totals per build, and the level passes of the last build by level and launch (the forest launches a
    level once per run of trees with the same code widths and node lookup)."""
    import csv
    with open(os.path.join(d, "forest", "run_kernel_trace.csv")) as f:
        rows = sorted(csv.DictReader(f), key=lambda r: int(r["Start_Timestamp"]))
    starts = [i for i, r in enumerate(rows) if _short_kernel(r["Kernel_Name"]) == "kf_init"]
    builds = []
    for b, i0 in enumerate(starts):
        i1 = starts[b + 1] if b + 1 < len(starts) else len(rows)
        seg = rows[i0:i1]
        g = [i for i, r in enumerate(seg) if _short_kernel(r["Kernel_Name"]) == "kf_gather"]
        builds.append(seg[:g[0] + 1] if g else seg)
    nb = len(builds)
    tot = {}
    for seg in builds:
        for r in seg:
            k = _short_kernel(r["Kernel_Name"])
            k = k if k.startswith("k_level") else k.split("<")[0]
            tot[k] = tot.get(k, 0.0) + (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
    last = builds[-1]
    span = (int(last[-1]["End_Timestamp"]) - int(last[0]["Start_Timestamp"])) / 1e3
    lines = ["# forest build graph (1024 u16 sequences, Σ n = 1.75·10^9): rocprofv3 kernel trace", "",
             "Command (repository root on the GPU box, `TMPDIR=/tmp`):", "", "    " + PROFILE_COMMANDS["forest"], "",
             "The run builds the forest %d times (warm-up included); every kernel node of the captured graph is its "
             "own dispatch. Last build: %d kernels, %.1f µs from the first kernel's start to the last one's end."
             % (nb, len(last), span), "", "Kernels of the graph, per build (mean over the run):", "",
             "| kernel | µs per build | % |", "|---|---|---|"]
    s_all = sum(tot.values())
    for k, v in sorted(tot.items(), key=lambda x: -x[1]):
        lines.append("| %s | %.1f | %.1f |" % (k, v / nb, 100.0 * v / s_all))
    lines += ["", "Level passes of the last build, µs per launch (E: element type of the level, EO: of the next "
              "level, kPos: nodes by position):", "", "| level | launch | blocks | µs |", "|---|---|---|---|"]
    lvl, per = -1, {}
    for r in last:
        k = _short_kernel(r["Kernel_Name"])
        if k == "kf_tile_reduce":
            lvl += 1
        if k.startswith("k_level"):
            us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            per[lvl] = per.get(lvl, 0.0) + us
            lines.append("| %d | %s | %d | %.1f |" % (lvl, k, int(r["Grid_Size_X"]) // int(r["Workgroup_Size_X"]), us))
    lines += ["", "Per level (all launches): " + ", ".join("%d: %.0f" % (l, v) for l, v in sorted(per.items())) +
              " µs; level passes %.1f µs in total." % sum(per.values()),
              "", "Source hash of the level kernel (sha256/16): %s." % source_hash(LEVEL_SRCS)]
    with open(os.path.join(out_dir, "forest_build_graph_trace.md"), "w") as f:
        f.write("\n".join(lines) + "\n")


# the rocprofv3 runs profile_summary reads (from the repository root; <out> is the directory it is given)
PROFILE_COMMANDS = {
    "trace": "rocprofv3 --kernel-trace --stats -f csv -d <out>/trace -o run -- python3 bench.py --no-cpu-baseline "
             "--no-extra > <out>/trace.json",
    "fetch": "rocprofv3 --pmc FETCH_SIZE -f csv -d <out>/fetch -o run -- python3 bench.py --steps 1 --warmup 0 "
             "--no-cpu-baseline --no-extra --calibrate-copy > <out>/fetch.json",
    "write": "rocprofv3 --pmc WRITE_SIZE -f csv -d <out>/write -o run -- python3 bench.py --steps 1 --warmup 0 "
             "--no-cpu-baseline --no-extra --calibrate-copy",
    "l2": "rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum -f csv -d <out>/l2 -o run -- python3 bench.py --steps 1 "
          "--warmup 0 --no-cpu-baseline --no-extra",
    "forest": "rocprofv3 --kernel-trace --stats -f csv -d <out>/forest -o run -- python3 bench.py --workload forest "
              "--steps 2 --warmup 1",
}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(name: str, n_sample: int, q_sample: int, runs: int = 3) -> dict:
    """The CPU oracle on a bounded prefix of the workload: every level's bits, directory and samples,
    then access/rank/select by sweeps, once on one thread and once on every host thread (OpenMP),
    median of `runs` runs each."""
    import oracle
    import workloads
    S, sigma = workloads.make_text(name, n=n_sample)
    qs = workloads.make_queries(name, S, sigma, q=q_sample)
    items = n_sample + 3 * q_sample

    def leg(nt):
        tb, tq = [], []
        for _ in range(runs):
            t0 = time.perf_counter()
            oracle.par_tree(S, sigma, nthreads=nt)
            t1 = time.perf_counter()
            oracle.par_access(S, qs["acc_pos"], nt)
            oracle.par_rank(S, sigma, qs["rank_c"], qs["rank_i"], nt)
            oracle.par_select(S, sigma, qs["sel_c"], qs["sel_k"], nt)
            t2 = time.perf_counter()
            tb.append(t1 - t0)
            tq.append(t2 - t1)
        tot = [a + b for a, b in zip(tb, tq)]
        return {"value": items / float(np.median(tot)), "threads": nt, "build_s_median": float(np.median(tb)),
                "queries_s_median": float(np.median(tq))}

    all_threads = oracle.par_threads(0)
    one = leg(1)
    many = leg(all_threads)
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {"value": many["value"], "unit": "(symbols+queries)/s", "cores": all_threads, "kind": "oracle",
            "sample": "first 2^%d symbols of the same text (every level's bits, rank directory and select samples, "
                      "one level per thread) + 2^%d access, rank and select queries drawn with the same recipe "
                      "(chunked sweeps over the text); median of %d runs"
                      % (n_sample.bit_length() - 1, q_sample.bit_length() - 1, runs),
            "single_thread": one, "all_threads": many, "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "affinity_cpus": affinity, "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def forest_level_bytes(f, w: int) -> float:
    """Algorithmic bytes of every level pass of every tree of a forest (as level_launch_bytes)."""
    return float(sum(sum(level_launch_bytes(t.info, w)) for t in f.trees))


def main_forest(args, torch, wt, workloads, dev):
    print(json.dumps(forest_leg(args, torch, wt, workloads, dev, args.steps, args.warmup, plain=True)), flush=True)


def forest_leg(args, torch, wt, workloads, dev, steps, warmup, plain):
    """The batched forest workload: `steps` timed forest builds plus mixed queries (after `warmup`), and
    with `plain` the same trees built and queried one at a time for comparison. Returns the JSON line."""
    cfg = workloads.FOREST
    print("# generating the batched workload (%d u16 sequences, %d mixed queries)" % (cfg["trees"], cfg["queries"]),
          file=sys.stderr, flush=True)
    fw = workloads.make_forest()
    n_total = int(fw.S.size)
    dS = torch.from_numpy(fw.S).to(dev)
    views = [dS[int(fw.offsets[j]):int(fw.offsets[j + 1])] for j in range(fw.trees)]
    sig = [int(x) for x in fw.sigmas]
    q = int(fw.arg.size)
    d_tree, d_op = torch.from_numpy(fw.tree).to(dev), torch.from_numpy(fw.op).to(dev)
    d_sym, d_arg = torch.from_numpy(fw.sym).to(dev), torch.from_numpy(fw.arg).to(dev)
    out = torch.empty(q, dtype=torch.uint64, device=dev)
    # the plain way: per tree and op, the query indexes (built once, outside the timed region)
    groups = []
    order = np.lexsort((fw.op, fw.tree))
    keys = fw.tree[order].astype(np.int64) * 4 + fw.op[order]
    bounds = np.searchsorted(keys, np.arange(fw.trees * 4 + 1))
    for j in range(fw.trees if plain else 0):
        g = []
        for o in range(3):
            idx = order[bounds[4 * j + o]:bounds[4 * j + o + 1]]
            g.append(None if idx.size == 0 else (torch.from_numpy(fw.sym[idx]).to(dev),
                                                  torch.from_numpy(fw.arg[idx]).to(dev),
                                                  torch.empty(idx.size, dtype=torch.uint64 if o else torch.uint32,
                                                              device=dev)))
        groups.append(g)
    del fw
    torch.cuda.synchronize()
    print("# autotuning |L2| and s per shape bucket", file=sys.stderr, flush=True)
    tune, trep = wt.autotune(views, sig)
    print("# tuned %d buckets in %.0f ms" % (trep["buckets"], trep["total_ms"]), file=sys.stderr, flush=True)

    def forest_step(record):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        t0 = time.perf_counter()
        f = wt.build_forest(views, sig, tune=tune)
        t1 = time.perf_counter()
        e0.record()
        f.query_mixed(d_tree, d_op, d_sym, d_arg, out=out)
        e1.record()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if record is not None:
            record.append(dict(build_s=t1 - t0, query_ms=e0.elapsed_time(e1), total_s=t2 - t0, info=dict(f.info),
                               level_bytes=forest_level_bytes(f, 2)))
        f.free()

    def plain_step():
        t0 = time.perf_counter()
        trees = [wt.build(v, s) for v, s in zip(views, sig)]
        t1 = time.perf_counter()
        for t, g in zip(trees, groups):
            if g[0] is not None:
                t.access(g[0][1], out=g[0][2])
            if g[1] is not None:
                t.rank(g[1][0], g[1][1], out=g[1][2])
            if g[2] is not None:
                t.select(g[2][0], g[2][1], out=g[2][2])
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for t in trees:
            t.free()
        return t1 - t0, t2 - t1, t2 - t0

    for _ in range(warmup):
        forest_step(None)
    recs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        forest_step(recs)
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / steps
    fb = float(np.median([r["build_s"] for r in recs]))
    fq = float(np.median([r["query_ms"] for r in recs])) * 1e-3
    gms = float(np.median([r["info"]["graph_ms"] for r in recs]))
    lb = recs[0]["level_bytes"]
    ach = lb / (gms * 1e-3) / 1e9
    line = {
        "metric": "batched build symbols/s + mixed queries/s (forest vs one tree at a time)",
        "value": (n_total + q) / (ms_per_step * 1e-3), "unit": "(symbols+queries)/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u16", "data": "synthetic",
        "config": {"workload": "forest", "trees": len(views), "symbols": n_total, "sym_bytes": 2,
                   "mixed_queries": q, "tuned_buckets": trep["buckets"]},
        "rates": {"forest_build_symbols_per_s": n_total / fb, "forest_build_ms": fb * 1e3,
                  "forest_graph_ms": gms, "forest_plan_ms": float(np.median([r["info"]["plan_ms"] for r in recs])),
                  "forest_capture_ms": float(np.median([r["info"]["capture_ms"] for r in recs])),
                  "forest_library_ms": float(np.median([r["info"]["total_ms"] for r in recs])),
                  "forest_graph_kernels": recs[0]["info"]["graph_kernels"],
                  "mixed_queries_per_s": q / fq, "mixed_ms": fq * 1e3},
        "roofline": {"kernel": "forest build graph (every level pass of every tree)", "bound": "hbm",
                     "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                     "traffic": None, "bytes_per_launch": lb, "avg_launch_ms": gms, "launches": len(recs),
                     "note": "level-pass algorithmic bytes of all trees / graph duration (includes histograms, "
                             "scans and node tables)"},
    }
    if plain:
        runs = [plain_step() for _ in range(max(1, min(steps, 3)))]
        pb, pq, pt = (float(np.median([p[i] for p in runs])) for i in range(3))
        line["rates"].update({"plain_build_symbols_per_s": n_total / pb, "plain_build_ms": pb * 1e3,
                              "plain_queries_per_s": q / pq, "plain_queries_ms": pq * 1e3,
                              "forest_vs_plain_build_speedup": pb / fb, "forest_vs_plain_query_speedup": pq / fq,
                              "forest_vs_plain_total_speedup": pt / (fb + fq)})
    return line


def main_serve(args, torch, wt, workloads, dev):
    T, N, QPOOL = 64, 1 << 26, 1 << 24
    print("# generating %d trees of 2^26 u8 Zipf(1.0)" % T, file=sys.stderr, flush=True)
    fw = workloads.make_forest(trees=T, n_range=(N, N), sigma_range=(256, 256), queries=0, width=1, index=4)
    dS = torch.from_numpy(fw.S).to(dev)
    views = [dS[int(fw.offsets[j]):int(fw.offsets[j + 1])] for j in range(T)]
    f = wt.build_forest(views, [256] * T)
    torch.cuda.synchronize()
    print("# query pool", file=sys.stderr, flush=True)
    base = workloads.subseed(workloads.base_seed(4), 1)
    r = [workloads.raw(workloads.subseed(base, k), 0, QPOOL) for k in range(4)]
    tree = (r[0] % np.uint64(T)).astype(np.uint32)
    pick = r[1] % np.uint64(10)
    op = np.where(pick < 7, 2, np.where(pick < 9, 1, 0)).astype(np.uint8)
    pos = r[2] % np.uint64(N)
    sym = fw.S[(fw.offsets[tree] + pos).astype(np.int64)].astype(np.uint32)
    arg = pos.copy()
    cnt = np.stack([np.bincount(fw.seq(j), minlength=256) for j in range(T)]).astype(np.uint64)
    sel = op == 2
    arg[sel] = 1 + r[3][sel] % cnt[tree[sel], sym[sel]]
    del fw, dS, views

    def pinned(a):
        t = torch.empty(a.size, dtype=getattr(torch, str(a.dtype)), pin_memory=True)
        t.numpy()[:] = a
        return t

    p_tree, p_op, p_sym, p_arg = pinned(tree), pinned(op), pinned(sym), pinned(arg)
    op_l = op.copy()
    op_l[op_l == 2] = 3
    p_op_l = pinned(op_l)
    p_out = torch.empty(QPOOL, dtype=torch.uint64, pin_memory=True)
    nreq = 2000
    sizes = workloads.loguniform(workloads.subseed(base, 5), nreq, 1, 1 << 20).astype(np.int64)
    offs = (workloads.raw(workloads.subseed(base, 6), 0, nreq) % np.uint64(QPOOL - (1 << 20))).astype(np.int64)
    u = workloads.raw(workloads.subseed(base, 7), 0, nreq).astype(np.float64) / 2.0 ** 64
    gaps = -np.log1p(-u)  # unit-mean exponential

    def requests(arrivals, learned):
        ops = p_op_l if learned else p_op
        rq = []
        for i in range(nreq):
            a, b = int(offs[i]), int(offs[i] + sizes[i])
            rq.append(dict(tree=p_tree[a:b], op=ops[a:b], sym=p_sym[a:b], arg=p_arg[a:b], out=p_out[a:b],
                           arrival_s=float(arrivals[i])))
        return rq

    def lat_stats(comps, st):
        lat = np.array([c["done_s"] - c["arrival_s"] for c in comps])
        small = sizes <= 16384
        d = {"qps": st["qps"], "p50_ms": st["lat_p50_s"] * 1e3, "p99_ms": st["lat_p99_s"] * 1e3,
             "p99_over_p50": st["lat_p99_s"] / max(st["lat_p50_s"], 1e-12), "batches": st["batches"],
             "peak_in_flight": st["peak_in_flight"], "peak_bytes": st["peak_bytes"]}
        wait = np.array([c["admit_s"] - c["arrival_s"] for c in comps])
        for name, m in (("small", small), ("large", ~small)):
            if m.any():
                d[name + "_p50_ms"] = float(np.percentile(lat[m], 50)) * 1e3
                d[name + "_p99_ms"] = float(np.percentile(lat[m], 99)) * 1e3
                # waiting for admission (a slot and budget) vs. from admission to completion
                d[name + "_wait_p99_ms"] = float(np.percentile(wait[m], 99)) * 1e3
                d[name + "_run_p99_ms"] = float(np.percentile((lat - wait)[m], 99)) * 1e3
        return d

    # the server as built (8 slots, small requests coalesced up to 16384 queries through page-locked
    # staging), and 4 slots or one request per batch for comparison; offered loads are fractions of the
    # first one's saturation rate
    res = {}
    sat_ref = None
    mean_q = float(sizes.mean())
    for key, slots, coalesce in (("coalesced_8_slots", 8, 0), ("coalesced_4_slots", 4, 0),
                                 ("per_request_8_slots", 8, 1)):
        srv = wt.Server(f, slots=slots, mem_budget=4 << 30, coalesce=coalesce)
        srv.run(requests(np.zeros(nreq), False)[:50])  # warm-up
        comps, sat = srv.run(requests(np.zeros(nreq), False))
        res[key] = {"slots": slots, "coalesce_q": coalesce or 16384, "saturation": lat_stats(comps, sat)}
        if sat_ref is None:
            sat_ref = sat["qps"]
        for rho in (0.5, 0.8, 0.95):
            lam = rho * sat_ref / mean_q  # batches/s
            arr = np.cumsum(gaps / lam)
            comps, st = srv.run(requests(arr, False))
            res[key]["rho%.2f" % rho] = lat_stats(comps, st)
        srv.close()
        print("# %s: %s" % (key, json.dumps(res[key])), file=sys.stderr, flush=True)
    f.free()
    line = {
        "metric": "serving queries/s with p50/p99 latency",
        "value": res["coalesced_8_slots"]["saturation"]["qps"], "unit": "queries/s", "n_gpus": 1, "steps": nreq, "warmup": 50,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "serve", "trees": T, "n_per_tree": N, "batches": nreq,
                   "batch_sizes": "log-uniform int [1, 2^20]", "mix": "70% select / 20% rank / 10% access",
                   "slots": 8, "coalesce_q": 16384, "mem_budget_bytes": 4 << 30, "host_buffers": "page-locked"},
        "rates": res,
        "note": "learned selects inside mixed batches are switched off (answered by the plain select)",
    }
    print(json.dumps(line), flush=True)


def run_bitvec(torch, wt, workloads, dev, n_bits: int, nq: int, reps: int = 3) -> dict:
    """Rank/select support of plain bit arrays (the thesis's rank/select benchmark): fill 10/50/90 %,
    uniform and adversarial placement of the ones, |L2| = 512, s = 16384; per array the build (event
    pair around wt_bv_build) and nq each of rank0, rank1, select0, select1 (positions uniform in
    [0, n_bits), k uniform in [1, count of b]); medians of `reps` timed runs after one warm-up."""
    l2, srate = 512, 16384
    base = workloads.subseed(workloads.base_seed(5), 0)
    pos = torch.from_numpy(workloads.uniform(workloads.subseed(base, 1), nq, n_bits)).to(dev)
    raw = torch.from_numpy((workloads.raw(workloads.subseed(base, 2), 0, nq) >> np.uint64(1)).astype(np.int64)).to(dev)
    out = torch.empty(nq, dtype=torch.uint64, device=dev)
    syms = [torch.full((nq,), b, dtype=torch.uint32, device=dev) for b in (0, 1)]
    stream = torch.cuda.current_stream()

    def timed(fn):
        ms = []
        for r in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            if r:
                ms.append(e0.elapsed_time(e1))
        return float(np.median(ms))

    res = {}
    wt.query_profiling(True)
    for dist in ("uniform", "adversarial"):
        for fill in (0.1, 0.5, 0.9):
            adv = dist == "adversarial"
            seed = workloads.subseed(base, 10 + 10 * int(adv) + int(round(fill * 10)))
            words = torch.from_numpy(workloads.bit_words(seed, n_bits, fill, adv)).to(dev)
            torch.cuda.synchronize()
            bl = []
            for rep in range(reps + 1):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                t = wt.build_bitvector(words, n_bits, l2_bits=l2, sample_rate=srate)
                e1.record(stream)
                torch.cuda.synchronize()
                if rep:
                    bl.append(e0.elapsed_time(e1))
                if rep < reps:
                    t.free()
            bms = float(np.median(bl))
            ones = t.info["level_ones"][0]
            cnt = {1: ones, 0: n_bits - ones}
            r = {"build_ms": bms, "ones": ones}
            kern = {}

            def kernels(key):
                # per-kernel time of the calls just timed (binning passes and traversal), mean per call
                acc = {}
                for e in wt.query_profile():
                    acc[e["kernel"]] = acc.get(e["kernel"], 0.0) + e["ms"] / (reps + 1)
                kern[key] = acc

            wt.query_profile()  # drop what the build left
            for b in (0, 1):
                r["rank%d_ms" % b] = timed(lambda: t.rank(syms[b], pos, out=out))
                kernels("rank%d" % b)
                k = (raw % max(cnt[b], 1) + 1).to(torch.uint64)
                r["select%d_ms" % b] = timed(lambda: t.select(syms[b], k, out=out))
                kernels("select%d" % b)
                del k
            for key in ("rank0", "rank1", "select0", "select1"):
                r[key + "_queries_per_s"] = nq / (r[key + "_ms"] * 1e-3)
            r["kernel_ms_per_call"] = kern
            r["build_bits_per_s"] = n_bits / (bms * 1e-3)
            res["%s_%d" % (dist, int(fill * 100))] = r
            t.free()
            del words
    # roofline of the slowest query kind: one 64-byte block of bits per query (random lines)
    worst = max(((k, q) for k, v in res.items() for q in ("rank0", "rank1", "select0", "select1")),
                key=lambda kq: res[kq[0]][kq[1] + "_ms"])
    wt.query_profiling(False)
    wms = res[worst[0]][worst[1] + "_ms"]
    ach = 64.0 * nq / (wms * 1e-3) / 1e9
    del pos, raw, out, syms
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return {"config": {"workload": "bitvec", "n_bits": n_bits, "queries_per_kind": nq, "l2_bits": l2,
                       "sample_rate": srate, "fills": [10, 50, 90], "placements": ["uniform", "adversarial"],
                       "runs": "median of %d after one warm-up" % reps},
            "arrays": res,
            "roofline_slowest": {"array": worst[0], "kind": worst[1], "bound": "hbm", "achieved": ach,
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                                 "note": "64 B (one L2 block of bits) per query, random lines"}}


def run_host_build(torch, wt, S_host, sigma, dev, chunk: int = 1 << 27, reps: int = 3) -> dict:
    """wt_build_host (the chunked build from host memory) from page-locked and pageable arrays, against
    copying the whole sequence to the device and building there (median host-clock ms of `reps` calls
    after one warm-up each)."""
    n = int(S_host.size)
    pin = torch.empty(n, dtype=getattr(torch, str(S_host.dtype)), pin_memory=True)
    pin.numpy()[:] = S_host
    res = {"n": n, "sym_bytes": int(S_host.dtype.itemsize), "chunk": chunk}
    for name, arr, two in (("pinned", pin.numpy(), False), ("pageable", S_host, False),
                           ("pinned_two_pass", pin.numpy(), True)):
        ms, cnt, bld, work = [], [], [], 0
        for r in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t, st = wt.build_host(arr, sigma, chunk=chunk, two_pass=two)
            t1 = time.perf_counter()
            t.free()
            if r:
                ms.append((t1 - t0) * 1e3)
                cnt.append(st["ms_counts"])
                bld.append(st["ms_build"])
                work = st["work_bytes"]
                res["chunks"] = st["chunks"]
                res[name + "_passes"] = st["passes"]
        res[name + "_ms"] = float(np.median(ms))
        res[name + "_counts_pass_ms"] = float(np.median(cnt))
        res[name + "_build_pass_ms"] = float(np.median(bld))
        res[name + "_symbols_per_s"] = n / (res[name + "_ms"] * 1e-3)
        res[name + "_work_bytes"] = int(work)
    cp, cb = [], []
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d = pin.to(dev, non_blocking=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        t = wt.build(d, sigma)
        t2 = time.perf_counter()
        t.free()
        del d
        if r:
            cp.append((t1 - t0) * 1e3)
            cb.append((t2 - t0) * 1e3)
    res["copy_ms"] = float(np.median(cp))
    res["copy_GB_per_s"] = n * res["sym_bytes"] / (res["copy_ms"] * 1e-3) / 1e9
    res["copy_then_device_build_ms"] = float(np.median(cb))
    res["pinned_vs_copy_then_build"] = res["copy_then_device_build_ms"] / res["pinned_ms"]
    del pin
    return res


def run_hostq(torch, wt, t, kinds, sizes, reps: int = 3) -> dict:
    """Queries from host memory (wt_query_host): for every query kind and batch size, the end-to-end time
    of the call (copies in, kernels, copies out) with page-locked and with pageable host arrays, beside
    the device-resident call on the same queries (median of `reps` after one warm-up; the first call of a
    page-locked configuration also builds its graph, which the warm-up absorbs)."""
    qmax = max(sizes)
    res = {}
    ops = {"access": wt.OP_ACCESS, "rank": wt.OP_RANK, "select": wt.OP_SELECT}
    stream = torch.cuda.current_stream()
    for kind, a in kinds.items():
        dsym, darg = (None, a[0]) if kind == "access" else (a[0], a[1])
        qk = min(qmax, darg.numel())
        arg_pg = darg[:qk].cpu().numpy().copy()
        sym_pg = None if dsym is None else dsym[:qk].cpu().numpy().copy()
        arg_pin = torch.from_numpy(arg_pg).pin_memory()
        sym_pin = None if sym_pg is None else torch.from_numpy(sym_pg).pin_memory()
        odt = np.uint32 if kind == "access" else np.uint64
        out_pg = np.zeros(qk, dtype=odt)
        out_pin = torch.zeros(qk, dtype=torch.uint32 if kind == "access" else torch.uint64).pin_memory()
        dout = torch.empty(qk, dtype=torch.uint32 if kind == "access" else torch.uint64, device=darg.device)
        for q in sizes:
            if q > qk:
                continue
            r = {}
            for mem in ("pinned", "pageable"):
                if mem == "pinned":
                    arg_h, sym_h, out_h = arg_pin[:q], None if sym_pin is None else sym_pin[:q], out_pin[:q]
                else:
                    arg_h, sym_h, out_h = arg_pg[:q], None if sym_pg is None else sym_pg[:q], out_pg[:q]
                ms = []
                for i in range(reps + 1):
                    t0 = time.perf_counter()
                    _, st = t.query_host(ops[kind], arg_h, sym_h, out=out_h)
                    t1 = time.perf_counter()
                    if i:
                        ms.append((t1 - t0) * 1e3)
                r[mem + "_ms"] = float(np.median(ms))
                r[mem + "_queries_per_s"] = q / (r[mem + "_ms"] * 1e-3)
                r[mem + "_chunks"] = st["chunks"]
                r[mem + "_graph"] = st["graph"]
            dms = []
            for i in range(reps + 1):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                if kind == "access":
                    t.access(darg[:q], out=dout[:q])
                elif kind == "rank":
                    t.rank(dsym[:q], darg[:q], out=dout[:q])
                else:
                    t.select(dsym[:q], darg[:q], out=dout[:q])
                e1.record(stream)
                torch.cuda.synchronize()
                if i:
                    dms.append(e0.elapsed_time(e1))
            r["device_resident_ms"] = float(np.median(dms))
            r["device_resident_queries_per_s"] = q / (r["device_resident_ms"] * 1e-3)
            r["pinned_vs_pageable_speedup"] = r["pageable_ms"] / r["pinned_ms"]
            res["%s_q%d" % (kind, q)] = r
            # the answers are those of the device-resident call
            ref = dout[:q].cpu().numpy()
            assert np.array_equal(out_pg[:q], ref) and np.array_equal(out_pin[:q].numpy(), ref), \
                "host-sourced %s differs from the device-resident answers" % kind
        del arg_pin, sym_pin, out_pin, dout
    wt.lib().wt_query_host_release()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="text_zipf")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the extra legs of the default run (matrix, Huffman, host memory, large alphabet, "
                         "forest, bit arrays)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned select index (training + queries)")
    ap.add_argument("--l2-bits", type=int, default=0, help="bits per L2 block (256..2048; 0: library default)")
    ap.add_argument("--sample-rate", type=int, default=0, help="select sample rate s (0: library default)")
    ap.add_argument("--bitvec-log2", type=int, default=32, help="bits of each array of the bit-array leg")
    ap.add_argument("--bitvec-queries", type=int, default=100_000_000, help="queries per kind of the bit-array leg")
    ap.add_argument("--hostq-max-log10", type=int, default=7,
                    help="largest host-sourced batch of the default run, 10^k queries (5..8)")
    ap.add_argument("--cpu-sample-log2", type=int, default=25)
    ap.add_argument("--cpu-queries-log2", type=int, default=20)
    ap.add_argument("--profile-summary", metavar="DIR",
                    help="write the summaries under profiles/ from the rocprofv3 runs kept in DIR, then exit")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (reference kernel for HBM counter scaling)")
    args = ap.parse_args()
    if args.profile_summary:
        profile_summary(args.profile_summary)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the wavelet-tree build and queries here run on a single MI355X "
              "(--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2505_03372_amd as wt
    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    wt.lib()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "forest":
        return main_forest(args, torch, wt, workloads, dev)
    if args.workload == "serve":
        return main_serve(args, torch, wt, workloads, dev)
    if args.workload == "bitvec":
        bv = run_bitvec(torch, wt, workloads, dev, 1 << args.bitvec_log2, args.bitvec_queries)
        worst = bv["roofline_slowest"]
        tot_ms = sum(r[k] for r in bv["arrays"].values() for k in r if k.endswith("_ms"))
        items = sum((1 << args.bitvec_log2) + 4 * args.bitvec_queries for _ in bv["arrays"])
        print(json.dumps({"metric": "bit-array build bits/s + rank/select queries/s", "value": items / (tot_ms * 1e-3),
                          "unit": "(bits+queries)/s", "n_gpus": 1, "steps": 3, "warmup": 1, "ms_per_step": tot_ms,
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
                          "data": "synthetic", "config": bv["config"], "arrays": bv["arrays"], "roofline": worst}),
              flush=True)
        return
    res = run_tree(args, torch, wt, workloads, dev, args.workload, args.steps, args.warmup,
                   learned=not args.no_learned, kinds_wanted=("access", "rank", "select"),
                   matrix_steps=0 if args.no_extra else 3,
                   hostq_sizes=() if args.no_extra else tuple(10 ** e for e in range(5, args.hostq_max_log10 + 1)),
                   host_build=not args.no_extra)
    n, width, sigma, q = res["n"], res["width"], res["sigma"], res["q"]
    ms_per_step = res["ms_per_step"]
    line = {
        "metric": "build symbols/s + access/rank/select queries/s; learned vs plain select",
        "value": res["items"] / (ms_per_step * 1e-3),
        "unit": "(symbols+queries)/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {1: "u8", 2: "u16", 4: "u32"}[width],
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "sym_bytes": width, "sigma": sigma, "queries_per_kind": q,
                   "query_kinds": res["kinds"], "l2_bits": res["info"]["l2_bits"],
                   "sample_rate": res["info"]["sample_rate"]},
        "rates": res["rates"],
        "roofline": res["roofline"],
        "roofline_build": res["roofline_build"],
        "roofline_build_total": res["roofline_build_total"],
    }
    if res["matrix"] is not None:
        line["matrix"] = res["matrix"]
    if res["huffman"] is not None:
        line["huffman"] = res["huffman"]
    if res["hostq"] is not None:
        line["host_queries"] = res["hostq"]
    if res["host_build"] is not None:
        line["host_build"] = res["host_build"]
    if args.workload == "text_zipf" and not args.no_extra:
        # the large-alphabet configuration (2^28 u32 symbols, sigma 2^20, 2^24 rank + 2^24 select), measured
        # in the same run after the main workload, outside its timed steps
        print("# large-alphabet leg", file=sys.stderr, flush=True)
        la = run_tree(args, torch, wt, workloads, dev, "large_alpha", 5, 2, learned=False,
                      kinds_wanted=("rank", "select"))
        line["large_alpha"] = {
            "config": {"workload": "large_alpha", "n": la["n"], "sym_bytes": la["width"], "sigma": la["sigma"],
                       "queries_per_kind": la["q"], "query_kinds": la["kinds"], "steps": 5, "warmup": 2},
            "ms_per_step": la["ms_per_step"], "value": la["items"] / (la["ms_per_step"] * 1e-3),
            "unit": "(symbols+queries)/s", "rates": la["rates"], "roofline": la["roofline"],
            "roofline_build": la["roofline_build"], "roofline_build_total": la["roofline_build_total"]}
    if args.workload == "text_zipf" and not args.no_extra:
        # the batched forest build (1024 u16 sequences) and its mixed queries, outside the timed steps
        print("# forest leg", file=sys.stderr, flush=True)
        fl = forest_leg(args, torch, wt, workloads, dev, 3, 1, plain=False)
        line["forest"] = {k: fl[k] for k in ("config", "ms_per_step", "value", "unit", "rates", "roofline")}
        torch.cuda.empty_cache()
    if args.workload == "text_zipf" and not args.no_extra:
        # the rank/select benchmark of plain bit arrays, outside the timed steps
        print("# bit-array leg", file=sys.stderr, flush=True)
        line["bitvec"] = run_bitvec(torch, wt, workloads, dev, 1 << args.bitvec_log2, args.bitvec_queries)
    if args.calibrate_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        line["calibration_copy_bytes"] = 1 << 30
        del src, dst
    if not args.no_cpu_baseline:
        print("# timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(args.workload, 1 << args.cpu_sample_log2, 1 << args.cpu_queries_log2)
    print(json.dumps(line), flush=True)


def run_tree(args, torch, wt, workloads, dev, name, steps, warmup, learned, kinds_wanted, matrix_steps=0,
             hostq_sizes=(), host_build=False):
    """Timed steps of one single-tree workload: build (+ learned-index training) + queries + free."""
    idx, n, width, sigma, q = workloads.CONFIGS[name]
    print("# generating workload %s: n=%d width=%d sigma=%d q=%d" % (name, n, width, sigma, q),
          file=sys.stderr, flush=True)
    wl = workloads.make(name, kinds=kinds_wanted)
    S = torch.from_numpy(wl.S).to(dev)
    kinds = {}
    if wl.acc_pos is not None:
        kinds["access"] = (torch.from_numpy(wl.acc_pos).to(dev),)
    if wl.rank_c is not None:
        kinds["rank"] = (torch.from_numpy(wl.rank_c).to(dev), torch.from_numpy(wl.rank_i).to(dev))
    if wl.sel_c is not None:
        kinds["select"] = (torch.from_numpy(wl.sel_c).to(dev), torch.from_numpy(wl.sel_k).to(dev))
    outs = {"access": torch.empty(q, dtype=torch.uint32, device=dev),
            "rank": torch.empty(q, dtype=torch.uint64, device=dev),
            "select": torch.empty(q, dtype=torch.uint64, device=dev),
            "select_learned": torch.empty(q, dtype=torch.uint64, device=dev)}
    S_host = wl.S if host_build else None
    del wl
    torch.cuda.synchronize()
    print("# workload resident in HBM", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    wt.query_profiling(True)
    use_learned = learned and "select" in kinds

    def step(record, shape="tree"):
        # the build is timed by one event pair around the whole wt_build call on its stream (it includes
        # the library's allocations, launch gaps and the final read-back of the level sizes) and by the
        # host wall time of the call; the per-kernel times come from separate builds with the library's
        # per-kernel events (each event pair leaves a gap of about 10 us on the stream)
        eb0, eb1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        eb0.record(stream)
        h0 = time.perf_counter()
        t = wt.build(S, sigma, l2_bits=args.l2_bits, sample_rate=args.sample_rate, matrix=shape == "matrix",
                     huffman=shape == "huffman")
        h1 = time.perf_counter()
        eb1.record(stream)
        evs = {}
        linfo = None
        if use_learned and shape == "tree":
            linfo = t.learn_select()
        for kind, a in kinds.items():
            for variant in (("plain", "learned") if kind == "select" and linfo is not None else ("plain",)):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                if kind == "access":
                    t.access(a[0], out=outs[kind])
                elif kind == "rank":
                    t.rank(a[0], a[1], out=outs[kind])
                elif variant == "plain":
                    t.select(a[0], a[1], out=outs[kind])
                else:
                    t.select_learned(a[0], a[1], out=outs["select_learned"])
                e1.record(stream)
                evs[kind if variant == "plain" else "select_learned"] = (e0, e1)
        qprof = wt.query_profile()  # per-kernel durations of this step's query calls (waits for them)
        if record is not None:
            record.append((None, evs, t.info, linfo, qprof, (eb0, eb1), (h1 - h0) * 1e3))
        t.free()

    def kernel_profiles(k, shape="tree"):
        # per-kernel durations of k builds made with the library's events (outside the timed steps)
        out = []
        for _ in range(k):
            t = wt.build(S, sigma, l2_bits=args.l2_bits, sample_rate=args.sample_rate, profile=True,
                         matrix=shape == "matrix", huffman=shape == "huffman")
            torch.cuda.synchronize()
            out.append(t.profile())
            t.free()
        return out

    for _ in range(warmup):
        step(None)
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        step(recs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wt.query_profiling(False)
    unbinned = None
    if use_learned:
        # Outside the timed steps: select in batches below the binning size (answered in input order,
        # so every level's reads land on random lines), where the learned index saves the node entry,
        # the samples and the L1 search that binned batches turn into shared cache hits.
        t = wt.build(S, sigma, l2_bits=args.l2_bits, sample_rate=args.sample_rate)
        t.learn_select()
        sc, sk = kinds["select"]
        nq, chunk = min(q, 1 << 24), 1 << 15
        unbinned = {"queries": nq, "batch": chunk}
        for variant, fn, out in (("plain", t.select, outs["select"]), ("learned", t.select_learned,
                                                                        outs["select_learned"])):
            for _ in range(2):  # the first pass warms up
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for i in range(0, nq, chunk):
                    fn(sc[i:i + chunk], sk[i:i + chunk], out=out[i:i + chunk])
                e1.record(stream)
                torch.cuda.synchronize()
            unbinned[variant + "_ms"] = e0.elapsed_time(e1)
        unbinned["learned_vs_plain_speedup"] = unbinned["plain_ms"] / unbinned["learned_ms"]
        t.free()
    ms_per_step = (t1 - t0) * 1e3 / steps
    profs = kernel_profiles(max(3, steps))
    hostq = None
    if hostq_sizes:
        t = wt.build(S, sigma, l2_bits=args.l2_bits, sample_rate=args.sample_rate)
        hostq = run_hostq(torch, wt, t, kinds, hostq_sizes)
        t.free()
    def shape_leg(shape, k_steps):
        # another shape of the same sequence answering the same queries (outside the timed steps)
        wt.query_profiling(True)
        step(None, shape)
        mrecs = []
        m0 = time.perf_counter()
        for _ in range(k_steps):
            step(mrecs, shape)
        torch.cuda.synchronize()
        m1 = time.perf_counter()
        wt.query_profiling(False)
        mprofs = kernel_profiles(k_steps, shape)
        res = {"steps": k_steps, "ms_per_step": (m1 - m0) * 1e3 / k_steps,
               "build_ms_median": float(np.median([r[5][0].elapsed_time(r[5][1]) for r in mrecs])),
               "build_kernel_sum_ms_median": float(np.median([sum(p["ms"] for p in pr) for pr in mprofs]))}
        res["build_symbols_per_s"] = n / (res["build_ms_median"] * 1e-3)
        inf = mrecs[0][2]
        res["levels"] = inf["levels"]
        res["level_bits_total"] = int(sum(inf["level_n"]))
        res["level_bits_per_symbol"] = res["level_bits_total"] / max(n, 1)
        mk = {}
        for r in mrecs:
            for k, (e0, e1) in r[1].items():
                res.setdefault(k + "_ms_median", []).append(e0.elapsed_time(e1))
            for e in r[4]:
                mk.setdefault(e["kernel"], []).append(e["ms"])
        for k in [k for k in res if k.endswith("_ms_median") and isinstance(res[k], list)]:
            res[k] = float(np.median(res[k]))
            res[k.replace("_ms_median", "_queries_per_s")] = q / (res[k] * 1e-3)
        for k, v in mk.items():
            res["kernel_%s_ms_per_step" % k] = float(np.sum(v)) / k_steps
        level = [p["ms"] for pr in mprofs for p in pr if p["kernel"] == "level"]
        res["build_level_kernel_ms_sum_median"] = float(np.median([sum(p["ms"] for p in pr if p["kernel"] == "level")
                                                                  for pr in mprofs])) if level else 0.0
        return res

    mat = shape_leg("matrix", matrix_steps) if matrix_steps else None
    huff = shape_leg("huffman", matrix_steps) if matrix_steps else None

    info = recs[0][2]
    level_ms, build_ms, build_ev_ms, build_wall_ms, learn_ms = [], [], [], [], []
    qms = {}
    kms = {}
    for prof in profs:
        level_ms += [p["ms"] for p in prof if p["kernel"] == "level"]
        build_ms.append(sum(p["ms"] for p in prof))
    for _, evs, _, linfo, qprof, (eb0, eb1), wall in recs:
        for e in qprof:
            kms.setdefault(e["kernel"], []).append(e["ms"])
        build_ev_ms.append(eb0.elapsed_time(eb1))
        build_wall_ms.append(wall)
        if linfo is not None:
            learn_ms.append(linfo["train_ms"])
        for k, (e0, e1) in evs.items():
            qms.setdefault(k, []).append(e0.elapsed_time(e1))
    per_launch = level_launch_bytes(info, width)
    avg_bytes = float(np.mean(per_launch))
    avg_ms = float(np.mean(level_ms))
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9
    items = n + q * len(qms)
    bms = float(np.median(build_ev_ms))
    rates = {"build_symbols_per_s": n / (bms * 1e-3)}
    for k in qms:
        rates[k + "_queries_per_s"] = q / (np.median(qms[k]) * 1e-3)
    rates["build_ms_median"] = bms
    rates["build_kernel_sum_ms_median"] = float(np.median(build_ms))
    rates["build_host_wall_ms_median"] = float(np.median(build_wall_ms))
    if learn_ms:
        rates["learn_train_ms_median"] = float(np.median(learn_ms))
        li = recs[0][3]
        rates["learned_models"] = li["models"]
        rates["learned_mean_err_blocks"] = li["mean_err_blocks"]
        rates["untrained_mean_err_blocks"] = li["mean_err_init_blocks"]
        rates["learned_vs_plain_select_speedup"] = float(np.median(qms["select"]) / np.median(qms["select_learned"]))
    if unbinned is not None:
        rates["select_unbinned"] = unbinned
    for k in qms:
        rates[k + "_ms_median"] = float(np.median(qms[k]))
    # kernels of the query calls: traversal kernels and the binning passes (per call, summed over kinds)
    for k, v in kms.items():
        per_call = float(np.sum(v)) / max(1, len(recs))
        rates["kernel_%s_ms_per_step" % k] = per_call
    kname = {1: "k_level<uint8_t>", 2: "k_level<uint16_t>", 4: "k_level<uint32_t>"}[width]
    build_roof = {"kernel": kname, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": achieved / HBM_PEAK_GBS,
                  "traffic": load_traffic(avg_bytes) if name == "text_zipf" else None,
                  "bytes_per_launch": avg_bytes, "avg_launch_ms": avg_ms, "launches": len(level_ms)}
    # the whole build (every kernel between the symbols on the device and the finished tree): one read
    # of the symbols for the histogram plus every level pass's bytes, over the event pair around wt_build
    # (frac) and over the sum of the kernels' own events (frac_kernel_sum)
    total_bytes = float(n * width + sum(per_launch))
    ksum = float(np.median(build_ms))
    build_total = {"bound": "hbm", "bytes": total_bytes, "ms": bms,
                   "achieved": total_bytes / (bms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": total_bytes / (bms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                   "ms_kernel_sum": ksum, "frac_kernel_sum": total_bytes / (ksum * 1e-3) / 1e9 / HBM_PEAK_GBS}
    # the kernel with the most time in a step: queries touch at least one 64-byte L2 block of bits per
    # level (random HBM lines), the level pass streams its level
    # the traversal kernel of each query kind, timed alone (events around the kernel on its stream)
    per_step = {k: float(np.median(kms[k])) for k in qms if k in kms}
    per_step["level"] = avg_ms * info["levels"]
    dom = max(per_step, key=per_step.get)
    if dom == "level":
        roof = build_roof
    else:
        blk = info["l2_bits"] // 8  # bytes of one L2 block of bits
        qbytes = float(blk) * info["levels"] * q
        qa = qbytes / (per_step[dom] * 1e-3) / 1e9
        roof = {"kernel": {"access": "k_access", "rank": "k_rank", "select": "k_select",
                           "select_learned": "k_select_learned"}[dom]
                          + "<%d, 1024u>" % (info["l2_bits"].bit_length() - 1),
                "bound": "hbm", "achieved": qa, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": qa / HBM_PEAK_GBS,
                "traffic": None, "bytes_per_launch": qbytes, "avg_launch_ms": per_step[dom], "launches": len(kms[dom]),
                "note": "random access: %d B (one L2 block of bits) per level per query" % blk}
        if name == "text_zipf":
            roof["traffic"] = load_query_traffic(roof["kernel"], q)
    del S, kinds, outs
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return {"n": n, "width": width, "sigma": sigma, "q": q, "kinds": list(qms.keys()), "info": info,
            "items": items, "ms_per_step": ms_per_step, "rates": rates, "roofline": roof,
            "roofline_build": build_roof, "roofline_build_total": build_total, "matrix": mat, "huffman": huff,
            "hostq": hostq, "host_build": run_host_build(torch, wt, S_host, sigma, dev) if host_build else None}


if __name__ == "__main__":
    main()
