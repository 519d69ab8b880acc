"""Benchmark: negacyclic polynomial product of two ciphertexts, N=2^16, L=24.

One step = forward NTT of 2 ciphertexts x 2 components x 24 limbs (96 NTTs),
pointwise product of the components (48), inverse NTT of the products (48),
all through libntt.so on one MI355X. Inputs are seeded synthetic residues,
resident in HBM before timing; the step rotates over buffer sets totalling
more than 1 GiB so each step reads data that is not in the 256 MB last-level
cache. Each timed step loop (one stream, then consecutive steps alternating
between two streams) runs --steady-ms of untimed steps first, then the
--warmup steps, then exactly --steps timed steps between two device
synchronisations. Prints one JSON line (metric, value in NTT/s, roofline of
the dominant kernel measured with HIP events, per-call baseline, CPU oracle
baseline, and the other sections' results).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0                 # MI355X HBM3E
INT32_MUL_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # 39.3: one int32 multiply per lane per clock
MULS_PER_SHOUP = 9                    # 32x32 products in one 64-bit Shoup product (approx quotient)
MULS_PER_GENERAL = 21                 # 32x32 products in one general 64-bit modular product
MULS_PER_MONT = 11                    # 32x32 products in one 64-bit Montgomery product (the fused product)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# sources that determine the timed kernels' machine code; counter-derived
# traffic is reported only while they are unchanged
KERNEL_SOURCES = ["paper_2405_11353_amd/csrc/ntt_core.hpp", "paper_2405_11353_amd/csrc/modarith.hpp",
                  "paper_2405_11353_amd/csrc/dispatch.inc", "paper_2405_11353_amd/csrc/k_u64.hip",
                  "paper_2405_11353_amd/csrc/k_u64w.hip", "paper_2405_11353_amd/csrc/k_pointwise.hip",
                  "paper_2405_11353_amd/csrc/launch.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "polymul_n65536_l24_traffic.json")
# rocprofv3 kernel names -> the names bench.py times them under
KERNEL_KEYS = [("k_col<nttk::Arith64<false, true>, 8, 16, true", "fwd_col_pass"),
               ("k_col<nttk::Arith64<false, false>, 8, 16, true", "fwd_col_pass"),
               ("k_row_st<nttk::Arith64<false, true>, 8, true", "fwd_row_pass"),
               ("k_row<nttk::Arith64<false, true>, 8, true, true", "fwd_row_pass"),
               ("k_row_st_inv<nttk::Arith64<false, false>, 8, true, true", "inv_row_pass_mul"),
               ("k_row_tw<nttk::Arith64<false, false>, 8, false, true, true", "inv_row_pass_mul"),
               ("k_row<nttk::Arith64<false, false>, 8, false, true, true", "inv_row_pass_mul"),
               ("k_col<nttk::Arith64<false, false>, 8, 16, false", "inv_col_pass"),
               ("k_pointwise<nttk::ModInfo64", "pointwise")]


HE_SOURCES = ["paper_2405_11353_amd/csrc/k_he.hip", "paper_2405_11353_amd/csrc/he.hpp",
              "paper_2405_11353_amd/csrc/modarith.hpp"]
HE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "he_keyswitch_n65536_traffic.json")
HE_KERNEL_KEYS = [("k_tensor<nttk::ModInfo64", "tensor_product"), ("k_bconv<8, 2, 8, false>", "mod_up"),
                  ("k_bconv<8, 2, 8, true>", "mod_down")]


def kernel_source_hash(files=None) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in files or KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def bench_key(name: str, keys=None):
    for pat, key in keys or KERNEL_KEYS:
        if pat in name:
            return key
    return None


def summarize_counters(d: str, he: bool = False):
    """Reads the rocprofv3 CSVs of one profiling session (kernel trace, FETCH_SIZE
    and WRITE_SIZE passes on bench.py and on the 1 GiB copy microbenchmark, SQ
    counters) from directory d and writes the summary files under profiles/
    (the NTT passes of the headline step, or with he=True the HE steps)."""
    import csv
    import collections
    import glob

    def pmc(sub):
        agg = collections.defaultdict(lambda: collections.defaultdict(list))
        for f in glob.glob(os.path.join(d, sub, "*counter_collection.csv")):
            for r in csv.DictReader(open(f)):
                agg[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
        return {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in agg.items()}

    if he:
        keys, sources, traffic_file = HE_KERNEL_KEYS, HE_SOURCES, HE_TRAFFIC_FILE
        md = os.path.join(ROOT, "profiles", "he_keyswitch_n65536_counters.md")
        title = ("# Counters and kernel trace: HE steps at N=2^16 (tensor product of 24-limb ciphertexts, "
                 "ModUp 3 x 8 -> 24 limbs, ModDown 2 x 8 -> 24 limbs), MI355X")
        B = "python3 bench.py --he-only"
    else:
        keys, sources, traffic_file = KERNEL_KEYS, KERNEL_SOURCES, TRAFFIC_FILE
        md = os.path.join(ROOT, "profiles", "polymul_n65536_l24_counters.md")
        title = "# Counters and kernel trace: polymul_n65536_l24 (N=2^16, 24 limbs, 2 ciphertexts), MI355X"
        B = ("python3 bench.py --steps 2 --warmup 1 --steady-ms 0 --kernel-reps 40 --streams 1 --no-cpu-baseline --no-per-call "
             "--no-batched --no-serving --no-paper-sizes --no-he --no-ablations --no-polymul --no-batch-sweep "
             "--no-latency")
    copy_f = [v["FETCH_SIZE"] for k, v in pmc("pmc_copy_fetch").items() if "k_copy" in k][0]
    copy_w = [v["WRITE_SIZE"] for k, v in pmc("pmc_copy_write").items() if "k_copy" in k][0]
    gib_kib = float(1 << 20)
    f_scale, w_scale = gib_kib / copy_f, gib_kib / copy_w
    fetch, write, sq = pmc("pmc_fetch"), pmc("pmc_write"), pmc("pmc_sq")
    # requests the L2 sends toward memory (the Infinity Cache sits behind this
    # interface, so a request counted here may still hit there), per kernel and
    # for the same 1 GiB copy
    dram = pmc("pmc_dram") if os.path.isdir(os.path.join(d, "pmc_dram")) else {}
    dcopy = pmc("pmc_copy_dram") if os.path.isdir(os.path.join(d, "pmc_copy_dram")) else {}
    dc = [v for k, v in dcopy.items() if "k_copy" in k]
    rd_per_gib = dc[0].get("TCC_EA0_RDREQ_DRAM_sum") if dc else None
    wr_per_gib = dc[0].get("TCC_EA0_WRREQ_DRAM_sum") if dc else None
    stats = {}
    for f in glob.glob(os.path.join(d, "kt", "*kernel_stats.csv")):
        for r in csv.DictReader(open(f)):
            stats[r["Name"]] = r
    out = {"source_hash": kernel_source_hash(sources), "fetch_scale": f_scale, "write_scale": w_scale,
           "kernels": {}}
    lines = [title, "",
             "Commands (run from the repository root on an MI355X; each pass is its own run):", "",
             f"    B='{B}'",
             "    rocprofv3 --kernel-trace --stats --output-format csv -d <dir>/kt -o kt -- $B",
             "    rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir>/pmc_fetch -o run -- $B",
             "    rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir>/pmc_write -o run -- $B",
             "    rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir>/pmc_copy_fetch -o run -- paper_2405_11353_amd/_build/ubench --copy-only",
             "    rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir>/pmc_copy_write -o run -- paper_2405_11353_amd/_build/ubench --copy-only",
             "    rocprofv3 --pmc SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_WAIT_INST_ANY SQ_WAVES --output-format csv -d <dir>/pmc_sq -o run -- $B"]
    if dram:
        lines += ["    rocprofv3 --pmc TCC_EA0_RDREQ_DRAM_sum TCC_EA0_WRREQ_DRAM_sum TCC_EA0_RDREQ_sum TCC_EA0_WRREQ_sum --output-format csv -d <dir>/pmc_dram -o run -- $B",
                  "    rocprofv3 --pmc TCC_EA0_RDREQ_DRAM_sum TCC_EA0_WRREQ_DRAM_sum TCC_EA0_RDREQ_sum TCC_EA0_WRREQ_sum --output-format csv -d <dir>/pmc_copy_dram -o run -- paper_2405_11353_amd/_build/ubench --copy-only"]
    lines += [f"    python3 bench.py --summarize-{'he-' if he else ''}counters <dir>", "",
             f"Scale factors from the plain copy of 1 GiB (read 1 GiB, write 1 GiB per dispatch): "
             f"FETCH_SIZE reads {copy_f:.0f} KiB -> x{f_scale:.3f}; WRITE_SIZE reads {copy_w:.0f} KiB -> x{w_scale:.3f}.",
             f"Kernel source hash: {out['source_hash']}", "",
             "| kernel | rocprof avg us | calls | scaled fetch MiB | scaled write MiB | VALU wave-instr | VALU busy | LDS bank conflicts | DRAM-bound reads (copy-scaled MiB) | DRAM-bound writes (copy-scaled MiB) |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    for name in sorted(set(fetch) | set(stats)):
        key = bench_key(name, keys)
        if key is None:
            continue
        avg_us = float(stats[name]["AverageNs"]) / 1e3 if name in stats else float("nan")
        calls = stats[name]["Calls"] if name in stats else "-"
        fb = fetch.get(name, {}).get("FETCH_SIZE", float("nan")) * 1024 * f_scale
        wb = write.get(name, {}).get("WRITE_SIZE", float("nan")) * 1024 * w_scale
        q = sq.get(name, {})
        valu = q.get("SQ_INSTS_VALU", float("nan"))
        busy = valu * 4 / (1024 * avg_us * 1e-6 * 2.4e9) if avg_us == avg_us else float("nan")
        dk = dram.get(name, {})
        dr = dk.get("TCC_EA0_RDREQ_DRAM_sum")
        dw = dk.get("TCC_EA0_WRREQ_DRAM_sum")
        dr_b = dr / rd_per_gib * (1 << 30) if dr is not None and rd_per_gib else None
        dw_b = dw / wr_per_gib * (1 << 30) if dw is not None and wr_per_gib else None
        out["kernels"][key] = {"rocprof_avg_us": avg_us, "fetch_bytes": fb, "write_bytes": wb,
                               "valu_wave_instr": valu, "lds_bank_conflicts": q.get("SQ_LDS_BANK_CONFLICT"),
                               "dram_read_bytes": dr_b, "dram_write_bytes": dw_b,
                               "dram_read_requests": dr, "dram_write_requests": dw}
        fmt = lambda v: f"{v / 2**20:.1f}" if v is not None else "-"  # noqa: E731
        lines.append(f"| {key} | {avg_us:.2f} | {calls} | {fb / 2**20:.1f} | {wb / 2**20:.1f} | {valu:.3g} | "
                     f"{busy:.0%} | {q.get('SQ_LDS_BANK_CONFLICT', float('nan')):.3g} | {fmt(dr_b)} | {fmt(dw_b)} |")
    lines += ["", "VALU busy = SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x avg duration x 2.4 GHz)."]
    if rd_per_gib:
        lines += ["DRAM-bound columns: TCC_EA0_RDREQ_DRAM_sum / TCC_EA0_WRREQ_DRAM_sum, requests the L2 sends toward "
                  f"memory, scaled by the same counters for the 1 GiB copy ({rd_per_gib:.4g} read and "
                  f"{wr_per_gib:.4g} write requests per GiB). The Infinity Cache sits behind that interface, so these "
                  "bound what reaches HBM from above; they cannot tell a hit there from HBM."]
    with open(traffic_file, "w") as fh:
        json.dump(out, fh, indent=1)
    with open(md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def counter_valu_busy(key: str):
    """VALU busy fraction of `key` from the stored counter summary
    (SQ_INSTS_VALU x 4 cycles over SIMDs x duration x 2.4 GHz), or None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    k = t.get("kernels", {}).get(key)
    if t.get("source_hash") != kernel_source_hash() or not k or not k.get("rocprof_avg_us"):
        return None
    return round(k["valu_wave_instr"] * 4 / (1024 * k["rocprof_avg_us"] * 1e-6 * 2.4e9), 3)


def counter_traffic(key: str, he: bool = False):
    """Scaled HBM bytes of one launch of `key` from the stored counter summary,
    or None if there is none or the kernel sources changed since."""
    try:
        with open(HE_TRAFFIC_FILE if he else TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash(HE_SOURCES if he else None) or key not in t.get("kernels", {}):
        return None
    k = t["kernels"][key]
    return round(k["fetch_bytes"] + k["write_bytes"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--streams", type=int, default=2,
                    help="streams that consecutive steps alternate between (1: all on one stream)")
    ap.add_argument("--steady-ms", type=float, default=200.0,
                    help="untimed steps for this long before the warm-up steps of each timed step loop (the "
                         "clocks ramp up under sustained load); 0 turns it off")
    ap.add_argument("--clock-warmup-ms", type=float, default=300.0,
                    help="device copies for this long before the per-kernel timing and before each later "
                         "section; 0 turns it off")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=3.0,
                    help="seconds per CPU-oracle leg (headline sample, all cores and one thread)")
    ap.add_argument("--no-per-call", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-latency", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-paper-sizes", action="store_true")
    ap.add_argument("--no-he", action="store_true")
    ap.add_argument("--no-ablations", action="store_true")
    ap.add_argument("--no-polymul", action="store_true")
    ap.add_argument("--he-only", action="store_true",
                    help="time only the HE steps (tensor product, ModUp, ModDown) and print their JSON")
    ap.add_argument("--summarize-he-counters", metavar="DIR", default=None,
                    help="write the HE-step counter summary under profiles/ from a rocprofv3 session")
    ap.add_argument("--serving-jobs", type=int, default=20000)
    ap.add_argument("--serving-warmup", type=int, default=1000)
    ap.add_argument("--no-batch-sweep", action="store_true")
    ap.add_argument("--polymul-only", action="store_true",
                    help="only the fused product (ntt_polymul) on one stream, --steps steps after --warmup")
    ap.add_argument("--summarize-roctx", metavar="DIR", default=None,
                    help="write profiles/roctx_ranges_polymul_n65536_l24.md from a marker trace of the headline run")
    ap.add_argument("--summarize-polymul-trace", metavar="DIR",
                    help="write profiles/polymul_fused_n65536_l24_trace.md from a kernel trace of --polymul-only")
    ap.add_argument("--serving-rate", type=float, default=15000.0,
                    help="offered load of the serving workload, jobs/s (Poisson arrivals)")
    ap.add_argument("--summarize-counters", metavar="DIR", default=None,
                    help="write profiles/ summaries from a rocprofv3 session directory and exit")
    return ap.parse_args()


def dist_us(xs) -> dict:
    """Mean, median, 99th percentile and minimum of per-run times (us)."""
    a = np.sort(np.asarray(xs, dtype=np.float64))
    return {"runs": int(a.size), "mean_us": round(float(a.mean()), 3), "p50_us": round(float(np.percentile(a, 50)), 3),
            "p99_us": round(float(np.percentile(a, 99)), 3), "min_us": round(float(a[0]), 3)}


def per_run_us(torch, fn, runs, stream):
    """Times of `runs` calls of fn(r), each between its own pair of HIP events
    on `stream` (the launch stream), in us."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(runs)]
    for r, (e0, e1) in enumerate(evs):
        e0.record(stream)
        fn(r)
        e1.record(stream)
    torch.cuda.synchronize()
    return [e0.elapsed_time(e1) * 1e3 for e0, e1 in evs]


_EXTRA_STREAMS = []


def extra_stream(torch, i):
    """The i-th stream beside the current one, created once and shared by every
    section that runs steps on several streams. HIP maps streams onto a few
    hardware queues (4 here) as they are created; a stream created late in a
    long run, after the library's and torch's other streams, can share a queue
    with the current stream, and work on the two then runs one after the other
    (measured: the fused product on two streams took 66 us per step with the
    pair the headline uses, 81-83 us with a stream created at the end of the
    full run)."""
    while len(_EXTRA_STREAMS) <= i:
        _EXTRA_STREAMS.append(torch.cuda.Stream())
    return _EXTRA_STREAMS[i]


def clock_warmup(torch, ms):
    """Device copies (1 GiB each way) for `ms` milliseconds before a timed
    section. From idle, the GPU's clocks ramp up over the first tens of
    milliseconds of sustained load, and drop again within half a second of
    idling. The copies are another kernel, so a kernel trace of the run holds
    only the timed kernels' own launches."""
    if ms <= 0:
        return
    a = torch.empty(128 << 20, dtype=torch.int64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < ms:
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
    del a, b


def bench_latency(ntt, si, torch, runs=200, warm=20):
    """The two small configurations, timed per call as the paper times its GPU
    runs (device-resident input and output, mean of at least 100 runs), with
    the median, 99th percentile and minimum beside the mean:
    single_ntt_n1024_u32 (one negacyclic NTT of 1024 32-bit words, q =
    998244353) and ciphertext_n16384_l8 (2 polynomials x 8 limbs of 2^14
    64-bit words, 16 transforms per call). Forward and inverse are timed
    apart, eagerly (events around each call) and replayed from a HIP graph
    that holds the one call. Each configuration's forward output is checked
    against the oracle first (the 1024-point one also against the O(N^2)
    definition), and every graph replay against the eager result."""
    import oracle
    stream = torch.cuda.current_stream()
    out = {}
    for w in (si.workload_single_u32(), si.workload_ct_n14()):
        flags = ntt.NTT_WORD32 if w.word == 32 else 0
        plan = ntt.Plan(w.N, w.moduli, flags=flags)
        host = si.poly_batch(w.seed, w.batch, w.moduli, w.N)
        as_dev = (lambda h: torch.from_numpy(h.astype(np.uint32).view(np.int32)).cuda()) if w.word == 32 else \
            (lambda h: torch.from_numpy(h.view(np.int64)).cuda())
        as_host = (lambda t: t.cpu().numpy().view(np.uint32).astype(np.uint64)) if w.word == 32 else \
            (lambda t: t.cpu().numpy().view(np.uint64))
        x = as_dev(host)
        chk = x.clone()
        plan.forward(chk)
        torch.cuda.synchronize()
        got = as_host(chk).reshape(host.shape)
        want = oracle.ntt_forward_batch(host, w.moduli)[0]
        assert (got == want).all(), f"{w.name}: forward differs from the oracle"
        if w.N <= 1024:
            assert (got[0, 0] == oracle.ntt_direct(host[0, 0], w.moduli[0])).all()
        plan.inverse(chk)
        torch.cuda.synchronize()
        assert torch.equal(chk, x), f"{w.name}: inverse(forward(x)) != x"
        n_ntt = w.batch * len(w.moduli)
        res = {"N": w.N, "L": len(w.moduli), "polys": w.batch, "word_bits": w.word, "ntts_per_call": n_ntt,
               "variant": list(ntt.ntt_plan_get_variant_for(plan.handle, w.batch))}
        for name, fn in (("forward", plan.forward), ("inverse", plan.inverse)):
            buf = x.clone()
            for _ in range(warm):
                fn(buf)
            eager = dist_us(per_run_us(torch, lambda r: fn(buf), runs, stream))
            # the same call captured once and replayed; any per-stream
            # workspace exists before the capture
            cs = torch.cuda.Stream()
            gbuf = x.clone()
            with torch.cuda.stream(cs):
                fn(gbuf, stream=cs)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=cs):
                fn(gbuf, stream=cs)
            ref = x.clone()
            gbuf.copy_(x)
            for rep in range(3):
                g.replay()
                fn(ref)
                torch.cuda.synchronize()
                assert torch.equal(gbuf, ref), f"{w.name} {name}: graph replay {rep} differs from the eager call"
            for _ in range(warm):
                g.replay()
            graph = dist_us(per_run_us(torch, lambda r: g.replay(), runs, stream))
            res[name] = {"eager": eager, "graph": graph,
                         "eager_ntt_per_s": round(n_ntt / (eager["mean_us"] * 1e-6), 1),
                         "graph_ntt_per_s": round(n_ntt / (graph["mean_us"] * 1e-6), 1)}
            log(f"latency {w.name} {name}: eager mean {eager['mean_us']:.2f} p50 {eager['p50_us']:.2f} "
                f"p99 {eager['p99_us']:.2f} min {eager['min_us']:.2f} us; graph mean {graph['mean_us']:.2f} "
                f"p50 {graph['p50_us']:.2f} p99 {graph['p99_us']:.2f} min {graph['min_us']:.2f} us")
            del g
        plan.close()
        out[w.name] = res
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(ntt, si, torch, host, base, step, seconds=3.0):
    """The CPU oracle (plain C, one 128-bit % per modular operation; a
    correctness reference, not a tuned CPU library) timed on this machine's
    host cores, on one thread and on all of them (OpenMP over independent
    (polynomial, limb) transforms), on bounded samples of each workload:
      polymul_n65536_l24: the headline step restricted to 4 of its 24 limbs
        (16 forward + 8 inverse NTTs + 8 products); its all-core rate is
        `value`, and the GPU's step output on that sample must equal it;
      single_ntt_n1024_u32: one 1024-point forward + inverse (32-bit words);
      ciphertext_n16384_l8: the whole configuration, 16 forward + 16 inverse;
      batched_uneven_256polys: forward transforms of the uneven batch (all
        256 polynomials on all cores, the first 16 on one thread).
    Each leg repeats its sample for about `seconds`."""
    import oracle
    w = si.workload_polymul_n16()
    moduli = w.moduli
    polys = host.shape[0]

    def rate(fn, ntts, nthreads, secs=seconds):
        done, t, used = 0, 0.0, 0
        while t < secs or done == 0:
            t0 = time.perf_counter()
            used = fn(nthreads)
            t += time.perf_counter() - t0
            done += ntts
        return round(done / t, 2), int(used), round(t, 2)

    legs = {}
    sub = 4
    ref_in = np.ascontiguousarray(host[:, :sub])
    last = {}

    def step_sample(nt):
        spec, used = oracle.ntt_forward_batch(ref_in, moduli[:sub], nthreads=nt)
        prod, _ = oracle.pointwise_batch(spec[:2], spec[2:], moduli[:sub], nthreads=nt)
        last["out"], _ = oracle.ntt_inverse_batch(prod, moduli[:sub], nthreads=nt)
        return used

    n_step = polys * sub + 2 * sub
    for key, nt in (("all_cores", 0), ("one_thread", 1)):
        v, used, t = rate(step_sample, n_step, nt)
        legs.setdefault(w.name, {})[key] = {"ntt_per_s": v, "threads": used, "seconds": t}
    legs[w.name]["sample"] = (f"the step restricted to limbs 0..{sub - 1}: {polys * sub} forward + {2 * sub} "
                              f"inverse NTTs + {2 * sub} pointwise products")
    gpu_buf = base.clone()
    step(gpu_buf)
    torch.cuda.synchronize()
    gpu_out = gpu_buf.cpu().numpy().view(np.uint64).reshape(host.shape)[:2, :sub]
    exact = bool((gpu_out == last["out"]).all())
    assert exact, "GPU result differs from the oracle on the CPU sample"

    w1 = si.workload_single_u32()
    x1 = si.poly_batch(w1.seed, 1, w1.moduli, w1.N)

    def single(nt):
        X, used = oracle.ntt_forward_batch(x1, w1.moduli, nthreads=nt)
        oracle.ntt_inverse_batch(X, w1.moduli, nthreads=nt)
        return used

    w2 = si.workload_ct_n14()
    x2 = si.poly_batch(w2.seed, w2.batch, w2.moduli, w2.N)

    def ct(nt):
        X, used = oracle.ntt_forward_batch(x2, w2.moduli, nthreads=nt)
        oracle.ntt_inverse_batch(X, w2.moduli, nthreads=nt)
        return used

    for wl, fn_, n in ((w1, single, 2), (w2, ct, 2 * w2.batch * len(w2.moduli))):
        legs[wl.name] = {}
        for key, nt in (("all_cores", 0), ("one_thread", 1)):
            v, used, t = rate(fn_, n, nt, secs=min(seconds, 1.5))
            legs[wl.name][key] = {"ntt_per_s": v, "threads": used, "seconds": t}
        legs[wl.name]["sample"] = "the whole configuration (forward + inverse)"

    jobs = si.batched_jobs()
    primes = si.batched_primes()
    s = si.Stream(si.BASE_SEED + 30)
    xs = [np.stack([s.uniform_mod(q, j.N) for q in primes[:j.L]])[None] for j in jobs]

    def batch_fwd(count):
        def run(nt):
            used = 0
            for j, x in zip(jobs[:count], xs[:count]):
                used = max(used, oracle.ntt_forward_batch(x, primes[:j.L], nthreads=nt)[1])
            return used
        return run

    legs["batched_uneven_256polys"] = {}
    for key, nt, count in (("all_cores", 0, len(jobs)), ("one_thread", 1, 16)):
        v, used, t = rate(batch_fwd(count), sum(j.L for j in jobs[:count]), nt, secs=0.0)
        legs["batched_uneven_256polys"][key] = {"ntt_per_s": v, "threads": used, "seconds": t, "polys": count}
    legs["batched_uneven_256polys"]["sample"] = "forward NTTs: all 256 polynomials on all cores, the first 16 on one thread"

    head = legs[w.name]
    res = {"value": head["all_cores"]["ntt_per_s"], "unit": "NTT/s", "cores": head["all_cores"]["threads"],
           "kind": "oracle", "sample": head["sample"] + f", repeated for {head['all_cores']['seconds']} s; "
                                                      "OpenMP over (poly, limb)",
           "value_one_thread": head["one_thread"]["ntt_per_s"], "cpu_model": cpu_model(),
           "nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
           "framing": "plain C correctness reference (one 128-bit % per modular operation), not a tuned CPU library",
           "gpu_matches_oracle_on_sample": exact, "workloads": legs}
    for name, lg in legs.items():
        log(f"cpu oracle {name}: {lg['all_cores']['ntt_per_s']:.1f} NTT/s on {lg['all_cores']['threads']} threads, "
            f"{lg['one_thread']['ntt_per_s']:.1f} NTT/s on 1 thread")
    return res


def bench_batched(ntt, si, torch, reps=10):
    """256 polynomials of uneven N (2^12..2^16) and limb count (1..32) in one
    hipGraph launch, against eager launches and one call per polynomial."""
    jobs = si.batched_jobs()
    primes = si.batched_primes()
    s = si.Stream(si.BASE_SEED + 30)
    tensors, hosts = [], []
    for j in jobs:
        x = np.stack([s.uniform_mod(q, j.N) for q in primes[:j.L]])
        hosts.append(x)
        tensors.append(torch.from_numpy(x.view(np.int64)).cuda())
    n_ntt = sum(j.L for j in jobs)
    words = sum(j.L * j.N for j in jobs)
    stream = torch.cuda.current_stream()
    fwd = ntt.Batch([(j.N, primes[:j.L], ntt.NTT_JOB_FORWARD, t) for j, t in zip(jobs, tensors)])
    inv = ntt.Batch([(j.N, primes[:j.L], ntt.NTT_JOB_INVERSE, t) for j, t in zip(jobs, tensors)])
    eager = ntt.Batch([(j.N, primes[:j.L], ntt.NTT_JOB_FORWARD, t) for j, t in zip(jobs, tensors)],
                      flags=ntt.NTT_BATCH_NO_GRAPH)
    serial = ntt.Batch([(j.N, primes[:j.L], ntt.NTT_JOB_FORWARD, t) for j, t in zip(jobs, tensors)],
                       flags=ntt.NTT_BATCH_SERIAL)
    import oracle
    # the oracle's forward of the first and last limb of every job
    chk_limbs = [sorted({0, j.L - 1}) for j in jobs]
    want = [oracle.ntt_forward_batch(np.ascontiguousarray(x[ls])[None], [primes[l] for l in ls])[0][0]
            for x, ls in zip(hosts, chk_limbs)]

    def check_forward(what):
        torch.cuda.synchronize()
        for i, (t, x, ls, w_) in enumerate(zip(tensors, hosts, chk_limbs, want)):
            got = t.cpu().numpy().view(np.uint64).reshape(x.shape)[ls]
            assert (got == w_).all(), f"{what}: job {i} differs from the oracle"

    def reload():
        for t, h in zip(tensors, hosts):
            t.copy_(torch.from_numpy(h.view(np.int64)))

    # exactness of the timed configuration: every job's forward output against
    # the oracle (first and last limb), then forward + inverse is the identity
    fwd.run()
    check_forward("graph batch")
    inv.run()
    torch.cuda.synchronize()
    exact = all(torch.equal(t, torch.from_numpy(h.view(np.int64)).cuda()) for t, h in zip(tensors, hosts))
    assert exact, "batched forward + inverse is not the identity"

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(n):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n * 1e3

    reload()
    serial.run()
    check_forward("graph batch with the buckets in sequence")
    # the three launch forms take turns over several rounds and each reports
    # its median round, so drift of the GPU's clock falls on all of them alike
    rounds = {"graph": [], "eager": [], "serial": []}
    for _ in range(5):
        rounds["graph"].append(timed(fwd.run, reps))
        rounds["eager"].append(timed(eager.run, reps))
        rounds["serial"].append(timed(serial.run, reps))
    us_graph, us_eager, us_serial = (float(np.median(rounds[k])) for k in ("graph", "eager", "serial"))
    # autotuned: every bucket size is tuned at its own item count, then the
    # batch is rebuilt (buckets pick their variants from the tuning table). The
    # process's table (the shipped one) is saved first and restored after, so
    # the sections that follow run with it.
    import tempfile
    saved_table = os.path.join(tempfile.mkdtemp(prefix="ntt_tune_"), "table.json")
    ntt.ntt_tune_save(saved_table)
    ntt.ntt_tune_clear()
    items_by_n = {}
    for j in jobs:
        items_by_n[j.N] = items_by_n.get(j.N, 0) + j.L
    choices = {}
    for N, items in sorted(items_by_n.items()):
        c = ntt.ntt_autotune(N, items=items, reps=5)
        choices[N] = {"items": items, "path": {2: "lds", 3: "fourstep"}.get(c["path"], c["path"]),
                      "log_n1": c["log_n1"], "exact": c["exact"], "us": round(c["us_per_call"], 1)}
    tuned = ntt.Batch([(j.N, primes[:j.L], ntt.NTT_JOB_FORWARD, t) for j, t in zip(jobs, tensors)])
    us_tuned = timed(tuned.run, reps)
    reload()
    tuned.run()
    check_forward("tuned batch")
    tuned.close()
    ntt.ntt_tune_clear()
    try:
        ntt.ntt_tune_load(saved_table)
    except ntt.NttError:
        pass  # the process had no table: defaults, as before the section
    os.remove(saved_table)
    os.rmdir(os.path.dirname(saved_table))
    plans = {}
    for j in jobs:
        if (j.N, j.L) not in plans:
            plans[(j.N, j.L)] = ntt.Plan(j.N, primes[:j.L])

    def per_call():
        for j, t in zip(jobs, tensors):
            plans[(j.N, j.L)].forward(t, batch=1)

    us_call = timed(per_call, max(2, reps // 2))
    info = fwd.info
    for b in (fwd, inv, eager, serial):
        b.close()
    for p_ in plans.values():
        p_.close()
    res = {"workload": "batched_uneven_256polys", "polys": len(jobs), "ntts": n_ntt, "coefficients": words,
           "graph_us": round(us_graph, 1), "graph_ntt_per_s": round(n_ntt / (us_graph * 1e-6), 1),
           "tuned_graph_us": round(us_tuned, 1), "tuned_ntt_per_s": round(n_ntt / (us_tuned * 1e-6), 1),
           "tuned_choices": choices,
           "graph_alg_GBs": round(16 * words / (us_graph * 1e-6) / 1e9, 1),
           "eager_us": round(us_eager, 1), "serial_graph_us": round(us_serial, 1),
           "rounds_us": {k: [round(t, 1) for t in v] for k, v in rounds.items()},
           "per_call_us": round(us_call, 1),
           "per_call_ntt_per_s": round(n_ntt / (us_call * 1e-6), 1),
           "graph_speedup_vs_per_call": round(us_call / us_graph, 2),
           "buckets": info["buckets"], "kernels": info["kernels"], "round_trip_exact": bool(exact),
           "checked": "forward of every job (first and last limb) vs the oracle, for the default and the tuned "
                      "batch; forward + inverse of every job is the identity"}
    log(f"batched: autotuned graph {us_tuned:.0f} us; choices {choices}")
    log(f"batched: {n_ntt} NTTs in {us_graph:.0f} us (graph of parallel branches), {us_serial:.0f} us (graph, buckets in sequence), {us_eager:.0f} us (eager), "
        f"{us_call:.0f} us (per-call) -> {res['graph_ntt_per_s'] / 1e6:.2f} M NTT/s")
    return res


# Table 1 of the paper: best FPGA latency per size (Pease_nc; 16 cores at
# 1K-16K, 4 cores at 64K), cyclic transform, 32-bit prime -- context only
PAPER_TABLE1_BEST_FPGA_US = {1024: 2.27, 4096: 8.60, 16384: 37.50, 65536: 669.30}


def graph_single(ntt, torch, plan, one, reps):
    """Mean time of one transform when `reps` dependent transforms are replayed
    from one captured HIP graph (launch overhead amortised), checked against
    the same transforms run eagerly, on two replays."""
    x0 = one.clone()
    buf = one.clone()
    cs = torch.cuda.Stream()
    with torch.cuda.stream(cs):
        plan.forward(buf, batch=1)     # any per-stream workspace exists before capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=cs):
        for _ in range(reps):
            plan.forward(buf, batch=1)
    ref = x0.clone()
    for rep in range(2):
        buf.copy_(x0) if rep == 0 else None
        g.replay()
        for _ in range(reps):
            plan.forward(ref, batch=1)
        torch.cuda.synchronize()
        assert torch.equal(buf, ref), "graph replay differs from the eager transforms"
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    return round(e0.elapsed_time(e1) / reps * 1e3, 3)


def bench_paper_sizes(ntt, si, torch, reps=100, batch=1024):
    """The paper's own setting: one cyclic transform with a 32-bit prime at
    1K/4K/16K/64K, timed as the mean of 100 runs between device-resident
    input and output (the paper's GPU methodology), plus batched throughput,
    for the library's kernels and for the paper's algorithm variants run as
    one kernel per stage (DIT, DIF, Pease, Pease_nc, Stockham). For the
    library's kernels the 100 runs are also replayed from one HIP graph
    (single_us_graph), which removes the per-launch overhead."""
    q = si.Q_SMALL
    stream = torch.cuda.current_stream()
    variants = [("fused", None), ("dit", ntt.NTT_PATH_PAPER_DIT), ("dif", ntt.NTT_PATH_PAPER_DIF),
                ("pease", ntt.NTT_PATH_PAPER_PEASE), ("pease_nc", ntt.NTT_PATH_PAPER_PEASE_NC),
                ("stockham", ntt.NTT_PATH_PAPER_STOCKHAM)]
    out = []
    for N in (1024, 4096, 16384, 65536):
        x = si.Stream(si.BASE_SEED + 50).uniform_mod(q, N).astype(np.uint32)
        one = torch.from_numpy(x.view(np.int32)).cuda()
        many = one.repeat(batch)
        row = {"N": N, "paper_table1_best_fpga_us": PAPER_TABLE1_BEST_FPGA_US[N]}
        for vname, path in variants:
            plan = ntt.Plan(N, [q], flags=ntt.NTT_CYCLIC | ntt.NTT_WORD32)
            if path is not None:
                plan.set_variant(path)
            res = {}
            for name, buf, b in (("single_us", one, 1), ("batched", many, batch)):
                plan.forward(buf, batch=b)
                plan.inverse(buf, batch=b)
                torch.cuda.synchronize()
                n = reps if b == 1 else max(5, reps // 10)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(n):
                    plan.forward(buf, batch=b)
                e1.record(stream)
                torch.cuda.synchronize()
                us = e0.elapsed_time(e1) / n * 1e3
                if b == 1:
                    res["single_us"] = round(us, 3)
                else:
                    res["batched_ntt_per_s"] = round(b / (us * 1e-6), 1)
            if path is None:
                res["single_us_graph"] = graph_single(ntt, torch, plan, one, reps)
            row[vname] = res
            plan.close()
        out.append(row)
        log(f"paper size N={N}: " + ", ".join(f"{v}: {row[v]['single_us']} us / {row[v]['batched_ntt_per_s'] / 1e6:.1f} M/s"
                                             for v, _ in variants) + f"; fused from a graph: {row['fused']['single_us_graph']} us")
    return {"workload": "cyclic_u32_q998244353_single_and_batched", "reps": reps, "batch": batch, "sizes": out}


def bench_batch_sweep(ntt, si, torch, reps=30):
    """The headline shape (N = 2^16, 24 limbs) at B = 1..32 polynomials per call,
    forward and inverse timed separately (HIP events, mean over reps dependent
    calls on buffers rotated over >= 1 GiB): how the fixed cost of a launch is
    amortised as the batch grows. Each call is 24 B transforms."""
    w = si.workload_polymul_n16()
    N, moduli, L = w.N, w.moduli, len(w.moduli)
    plan = ntt.Plan(N, moduli)
    stream = torch.cuda.current_stream()
    host = si.poly_batch(w.seed, 1, moduli, N)
    one = torch.from_numpy(host.view(np.int64)).cuda()
    rows = []
    for B in (1, 2, 4, 8, 16, 32):
        base = one.repeat(B, 1, 1).contiguous()
        n_sets = max(2, math.ceil((1 << 30) / (base.numel() * 8)))
        sets = [base.clone() for _ in range(n_sets)]
        chk = base.clone()
        plan.forward(chk, batch=B)
        plan.inverse(chk, batch=B)
        torch.cuda.synchronize()
        assert torch.equal(chk, base), "batch sweep round trip is not exact"
        row = {"polys": B, "ntts_per_call": B * L}
        for name, fn in (("forward", plan.forward), ("inverse", plan.inverse)):
            for r in range(3):
                fn(sets[r % n_sets], batch=B)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for r in range(reps):
                fn(sets[r % n_sets], batch=B)
            e1.record(stream)
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) / reps * 1e3
            row[name + "_us"] = round(us, 1)
            row[name + "_ntt_per_s"] = round(B * L / (us * 1e-6), 1)
        rows.append(row)
        log(f"batch sweep B={B}: forward {row['forward_us']} us ({row['forward_ntt_per_s'] / 1e6:.2f} M NTT/s), "
            f"inverse {row['inverse_us']} us ({row['inverse_ntt_per_s'] / 1e6:.2f} M NTT/s)")
        del sets, base
    plan.close()
    return {"workload": w.name, "limbs": L, "N": N, "rows": rows}


def bench_polymul(ntt, si, torch, steps=100, warm=10, stream_counts=(1, 2), steady_ms=200.0):
    """The headline product (2 ciphertexts, N = 2^16, 24 limbs) through
    ntt_polymul, which keeps the spectra on chip: c = a * b for the 2 pairs of
    components, coefficients in and out. Reported per step and as the
    equivalent NTT rate (the same 96 forward and 48 inverse transforms), on one
    and on two streams, beside the headline step that hands the spectra back."""
    w = si.workload_polymul_n16()
    N, moduli, L = w.N, w.moduli, len(w.moduli)
    host = si.poly_batch(w.seed, 4, moduli, N)
    base = torch.from_numpy(host.view(np.int64)).cuda()
    n_sets = max(2, math.ceil((1 << 30) / (base.numel() * 8 * 3 // 2)))
    n_sets += n_sets % 2
    sets = [(base.clone(), torch.zeros_like(base[:2])) for _ in range(n_sets)]
    plan = ntt.Plan(N, moduli)
    stream = torch.cuda.current_stream()
    # check: equal to the unfused product
    ref = base.clone()
    plan.forward(ref, batch=4)
    plan.pointwise_inverse(ref[:2], ref[2:], ref[:2], batch=2)
    out = torch.zeros_like(base[:2])
    plan.polymul(base[:2], base[2:], out, batch=2)
    torch.cuda.synchronize()
    assert torch.equal(out, ref[:2]), "fused product differs from the unfused one"
    res = {"workload": w.name, "products_per_step": 2 * L, "ntt_equivalent_per_step": 144}
    for n_streams in stream_counts:
        sts = [stream] + [extra_stream(torch, i) for i in range(n_streams - 1)]
        # as for the headline step: untimed steps for steady_ms, then the warm-up
        t_st, r = time.perf_counter(), 0
        while (time.perf_counter() - t_st) * 1e3 < steady_ms:
            for _ in range(32):
                x, c = sets[r % n_sets]
                plan.polymul(x[:2], x[2:], c, batch=2, stream=sts[r % n_streams])
                r += 1
            torch.cuda.synchronize()
        for s in range(warm):
            x, c = sets[s % n_sets]
            plan.polymul(x[:2], x[2:], c, batch=2, stream=sts[s % n_streams])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for st in sts[1:]:
            st.wait_event(e0)
        for s in range(steps):
            x, c = sets[s % n_sets]
            plan.polymul(x[:2], x[2:], c, batch=2, stream=sts[s % n_streams])
        for st in sts[1:]:
            done = torch.cuda.Event()
            done.record(st)
            stream.wait_event(done)
        e1.record(stream)
        torch.cuda.synchronize()
        us = (time.perf_counter() - t0) * 1e6 / steps
        res[f"streams_{n_streams}"] = {"us_per_step": round(us, 1), "ntt_equivalent_per_s": round(144 / (us * 1e-6), 1)}
        log(f"polymul (spectra on chip), {n_streams} stream(s): {us:.1f} us/step, "
            f"{144 / (us * 1e-6) / 1e6:.3f} M NTT-equivalent/s")
    return res


def bench_ablations(ntt, si, torch, steps=100, warm=5):
    """The headline step (2 ciphertexts, N = 2^16, 24 limbs, one stream) with one
    design choice changed at a time: the row pass with the merged per-row
    twiddles instead of the twisted one, the four-step split N1 x N2, the
    exact quotient of the 64-bit Shoup product instead of the approximate one,
    and the pointwise product as its own pass instead of fused into the first
    inverse pass.
    Each variant is checked: forward then inverse returns the input."""
    w = si.workload_polymul_n16()
    N, moduli, L = w.N, w.moduli, len(w.moduli)
    host = si.poly_batch(w.seed, 4, moduli, N)
    base = torch.from_numpy(host.view(np.int64)).cuda()
    set_bytes = base.numel() * 8
    n_sets = max(2, math.ceil((1 << 30) / set_bytes))
    sets = [base.clone() for _ in range(n_sets)]
    stream = torch.cuda.current_stream()

    second = extra_stream(torch, 0)

    def make_step(plan, fused):
        def step(buf, st=None):
            plan.forward(buf, batch=4, stream=st)
            a, b = buf[:2], buf[2:]
            if fused:
                plan.pointwise_inverse(a, b, a, batch=2, stream=st)
            else:
                plan.pointwise(a, b, a, batch=2, stream=st)
                plan.inverse(a, batch=2, stream=st)
        return step

    def timed(step, n):
        for s in range(warm):
            step(sets[s % n_sets])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for s in range(n):
            step(sets[s % n_sets])
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n * 1e3

    def timed_two_streams(step, n):
        # consecutive steps alternate between two streams, as in the headline;
        # wall clock between two device synchronisations
        sts = [stream, second]
        for s in range(warm):
            step(sets[s % n_sets], sts[s % 2])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(n):
            step(sets[s % n_sets], sts[s % 2])
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n * 1e6

    TW = ntt.NTT_ROW_TWIST_FWD | ntt.NTT_ROW_TWIST_INV
    variants = [
        ("default: split 2^8 x 2^8, approximate quotient, fused product, twisted (split-twist) rows both ways",
         8, False, True, TW),
        ("merged-twiddle row passes", 8, False, True, 0),
        ("merged forward rows, twisted inverse rows", 8, False, True, ntt.NTT_ROW_TWIST_INV),
        ("split 2^7 x 2^9", 7, False, True, TW),
        ("split 2^9 x 2^7", 9, False, True, TW),
        ("exact quotient", 8, True, True, TW),
        ("separate pointwise pass", 8, False, False, TW)]
    plans, steps_of = [], []
    for name, log_n1, exact, fused, twist in variants:
        plan = ntt.Plan(N, moduli)
        plan.set_variant(ntt.NTT_PATH_FOURSTEP, log_n1)
        plan.set_exact_quotient(exact)
        plan.set_row_twist(twist)
        chk = base.clone()
        plan.forward(chk, batch=4)
        plan.inverse(chk, batch=4)
        torch.cuda.synchronize()
        assert torch.equal(chk, base), "ablation variant is not exact"
        plans.append(plan)
        steps_of.append(make_step(plan, fused))
    # the variants take turns, round after round, and each reports its median
    # round: drift of the GPU's speed during the section then falls on all alike
    rounds = 5
    # the row forms are also timed on two streams, where the headline runs and
    # where they differ (the split-twist rows read fewer table bytes)
    two = 3
    times = [[] for _ in variants]
    times2 = [[] for _ in variants[:two]]
    for _ in range(rounds):
        for i, step in enumerate(steps_of):
            times[i].append(timed(step, max(1, steps // rounds)))
            if i < two:
                times2[i].append(timed_two_streams(step, max(2, steps)))
    rows = []
    for i, ((name, log_n1, exact, fused, twist), ts) in enumerate(zip(variants, times)):
        us = float(np.median(ts))
        row = {"variant": name, "log_n1": log_n1, "exact_quotient": exact, "fused_product": fused,
               "row_twist_mask": twist, "us_per_step": round(us, 1), "ntt_per_s": round(144 / (us * 1e-6), 1),
               "rounds_us": [round(t, 1) for t in ts]}
        msg = f"ablation {name}: {us:.1f} us/step"
        if i < two:
            us2 = float(np.median(times2[i]))
            row.update({"us_per_step_two_streams": round(us2, 1), "rounds_two_streams_us": [round(t, 1) for t in times2[i]]})
            msg += f", {us2:.1f} us/step on two streams"
        rows.append(row)
        log(msg + f" (medians of {rounds} interleaved rounds)")
    for plan in plans:
        plan.close()
    return {"workload": w.name, "streams": 1, "rounds": rounds, "rows": rows}


def bench_he_steps(ntt, si, torch, reps=50):
    """The HE steps around the transform at the headline shape (N = 2^16, 24
    ciphertext limbs of 60 bits) with 8 special primes and 3 key-switching
    digits of 8 limbs: the tensor product of one ciphertext pair, ModUp of
    the 3 digits (8 -> 24 limbs: the other 16 ciphertext limbs and the 8
    special primes) and ModDown of the 2 key-switching outputs (8 special
    limbs -> 24 limbs). Each kernel rotates over buffer sets larger than the
    last-level cache and is timed with HIP events on its launch stream."""
    N, L, K_sp, digit = 1 << 16, 24, 8, 8
    primes = si.ntt_primes(60, 17, L + K_sp)
    q, p = primes[:L], primes[L:]
    stream = torch.cuda.current_stream()
    plan = ntt.Plan(N, q)
    modup = ntt.BaseConv(N, q[:digit], q[digit:] + p)      # one digit; the others use their own plan
    moddown = ntt.BaseConv(N, p, q)
    words = lambda n: torch.zeros(n, dtype=torch.int64, device="cuda")   # noqa: E731

    def sets_for(nbytes):
        return max(2, math.ceil((512 << 20) / nbytes))

    def fill(t, moduli, seed):
        per = N * len(moduli)
        host = si.poly_batch(seed, t.numel() // per, moduli, N)
        t.copy_(torch.from_numpy(host.reshape(-1).view(np.int64)))
        return t

    def timed(fn, n_sets):
        for r in range(3):
            fn(r % n_sets)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for r in range(reps):
            fn(r % n_sets)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e3

    def entry(us, nbytes, muls):
        gbs = nbytes / (us * 1e-6) / 1e9
        tops = muls / (us * 1e-6) / 1e12
        return dict(us=round(us, 2), alg_bytes=nbytes, hbm_GBs=round(gbs, 1), hbm_frac=round(gbs / HBM_PEAK_GBS, 4),
                    alg_int32_muls=muls, mul_TOPs=round(tops, 3), mul_frac=round(tops / INT32_MUL_PEAK_TOPS, 4))

    out = {"workload": "he_keyswitch_n65536_l24_k8_dnum3", "N": N, "L": L, "special_primes": K_sp, "digits": 3}
    # tensor product: read 4 words, write 3 per (limb, coefficient); 4 general products
    tb = 7 * L * N * 8
    ns = sets_for(tb)
    A = [fill(words(2 * L * N), q * 2, 700 + i) for i in range(ns)]
    B = [fill(words(2 * L * N), q * 2, 800 + i) for i in range(ns)]
    D = [words(3 * L * N) for _ in range(ns)]
    us = timed(lambda i: plan.tensor_product(A[i], B[i], D[i], batch=1), ns)
    out["tensor_product"] = entry(us, tb, 4 * L * N * MULS_PER_GENERAL)
    del A, B, D
    # ModUp: 3 digits of 8 limbs -> 24 limbs; the dot products take 4
    # 32x32 multiplies per (source, target) pair and coefficient
    ub = 3 * (digit + L) * N * 8
    ns = sets_for(ub)
    X = [fill(words(3 * digit * N), q[:digit], 900 + i) for i in range(ns)]
    Y = [words(3 * L * N) for _ in range(ns)]
    us = timed(lambda i: modup.convert(X[i], Y[i], batch=3), ns)
    out["mod_up"] = entry(us, ub, 3 * N * digit * L * 4)
    del X, Y
    # ModDown: 2 polynomials, read 8 special + 24 limbs, write 24
    db = 2 * (K_sp + 2 * L) * N * 8
    ns = sets_for(db)
    X = [fill(words(2 * K_sp * N), p, 1000 + i) for i in range(ns)]
    Y = [fill(words(2 * L * N), q, 1100 + i) for i in range(ns)]
    us = timed(lambda i: moddown.mod_down(X[i], Y[i], Y[i], batch=2), ns)
    out["mod_down"] = entry(us, db, 2 * N * K_sp * L * 4)
    del X, Y
    for k in ("tensor_product", "mod_up", "mod_down"):
        e = out[k]
        e["traffic"] = counter_traffic(k, he=True)
        log(f"he {k}: {e['us']:.1f} us  {e['hbm_GBs']:.0f} GB/s ({e['hbm_frac']:.1%} HBM)  "
            f"{e['mul_TOPs']:.2f} TOP/s int32 mul ({e['mul_frac']:.1%})")
    return out


def bench_serving(ntt, si, torch, n_jobs=20000, warm=1000, rate=15000.0):
    """Poisson stream of NTT and poly-mult jobs (N 2^12..2^17, L 1..40) at a fixed
    offered load through the server, against a per-call FIFO; the saturated
    rate of a queued burst is reported beside it."""
    import threading
    primes = si.serving_primes()
    s = si.Stream(si.BASE_SEED + 40)
    logns = range(12, 18)
    pool_a = {}
    pool_b = {}
    for lg in logns:
        N = 1 << lg
        a = np.stack([s.uniform_mod(q, N) for q in primes])
        b = np.stack([s.uniform_mod(q, N) for q in primes])
        pool_a[lg] = torch.from_numpy(a.view(np.int64)).cuda()
        pool_b[lg] = torch.from_numpy(b.view(np.int64)).cuda()
    ring = [torch.empty(40 << 17, dtype=torch.int64, device="cuda") for _ in range(64)]

    def job_args(i, j):
        lg = j.N.bit_length() - 1
        op = ntt.NTT_REQ_POLYMUL if j.op == "polymul" else ntt.NTT_REQ_NTT
        a = pool_a[lg][:j.L]
        b = pool_b[lg][:j.L] if op == ntt.NTT_REQ_POLYMUL else None
        return op, j.N, primes[:j.L], a, ring[i % len(ring)], b

    def ntts_of(j):
        return j.L * (3 if j.op == "polymul" else 1)

    server = ntt.Server(hbm_budget_bytes=4 << 30, n_streams=4, max_batch_items=4096)

    def prepare(jobs):
        out = []
        for i, j in enumerate(jobs):
            op, N, mods, a, o, b = job_args(i, j)
            out.append(server.make_request(op, N, mods, a, o, b))
        return out

    # saturated throughput: a burst of jobs, all queued at once (requests are
    # prepared beforehand so the submit loop is the C call only)
    burst = si.serving_trace(seed=si.BASE_SEED + 41, count=2000)
    reqs = prepare(burst)
    # one job per length over all the primes, and the burst's first jobs: every
    # (q, N) twiddle table the server will use is built before any timing
    for lg in logns:
        wa = ring[0][:len(primes) << lg].view(len(primes), 1 << lg)
        r = server.make_request(ntt.NTT_REQ_POLYMUL, 1 << lg, primes, pool_a[lg], wa, pool_b[lg])
        assert server.wait(server.submit_request(r)) == 0
    for r in reqs[:50]:
        assert server.wait(server.submit_request(r)) == 0
    t0 = time.perf_counter()
    tk = [server.submit_request(r) for r in reqs]
    for t in tk:
        assert server.wait(t) == 0
    sat_jobs_s = len(burst) / (time.perf_counter() - t0)
    def replay_server(trace, treqs):
        server.reset_stats()
        tickets = []
        start = time.perf_counter()
        for i, j in enumerate(trace):
            while time.perf_counter() - start < j.arrival_s:
                pass
            tickets.append(server.submit_request(treqs[i]))
            if i == warm - 1:
                server.reset_stats()
        for t in tickets:
            assert server.wait(t) == 0
        return time.perf_counter() - start

    # latency against offered load: the same job mix at fractions of the burst rate
    curve = []
    for frac in (0.3, 0.5, 0.7):
        r = frac * sat_jobs_s
        tr = si.serving_trace(seed=si.BASE_SEED + 42, count=warm + n_jobs, rate_per_s=r)
        replay_server(tr, prepare(tr))
        cs = server.stats()
        curve.append({"offered_jobs_per_s": round(r, 1), "fraction_of_burst_rate": frac,
                      "p50_us": round(cs["p50_us"], 1), "p99_us": round(cs["p99_us"], 1),
                      "mean_jobs_per_batch": round(cs["completed"] / max(1, cs["batches"]), 2),
                      "jobs_measured": cs["completed"], "ntt_per_s": round(cs["ntts"] / max(cs["wall_s"], 1e-9), 1),
                      "max_inflight_batches": cs["max_inflight_batches"]})
        log(f"serving at {r:.0f} jobs/s ({frac:.0%} of the burst rate): p50 {curve[-1]['p50_us']} us "
            f"p99 {curve[-1]['p99_us']} us, {curve[-1]['mean_jobs_per_batch']} jobs per batch")

    trace = si.serving_trace(count=warm + n_jobs, rate_per_s=rate)
    treqs = prepare(trace)
    wall = replay_server(trace, treqs)
    st = server.stats()
    server.close()

    # the 70%-of-burst trace under other HBM budgets: admission holds jobs whose
    # working memory does not fit beside the jobs in flight
    budgets = []
    hi = si.serving_trace(seed=si.BASE_SEED + 42, count=warm + n_jobs, rate_per_s=0.7 * sat_jobs_s)
    # (the job mix's 240 (q, N) table sets take 315 MiB of any budget)
    for gib in (0.5, 1, 4, 16):
        server = ntt.Server(hbm_budget_bytes=int(gib * (1 << 30)), n_streams=4, max_batch_items=4096)
        replay_server(hi, prepare(hi))
        bs = server.stats()
        server.close()
        budgets.append({"hbm_budget_GiB": gib, "offered_jobs_per_s": round(0.7 * sat_jobs_s, 1), "p50_us": round(bs["p50_us"], 1), "p99_us": round(bs["p99_us"], 1),
                        "admission_stalls": bs["admission_stalls"],
                        "max_inflight_batches": bs["max_inflight_batches"],
                        "mean_jobs_per_batch": round(bs["completed"] / max(1, bs["batches"]), 2),
                        "peak_bytes": bs["peak_bytes"], "table_bytes": bs["table_bytes"],
                        "table_uploads": bs["table_uploads"], "table_evictions": bs["table_evictions"]})
        log(f"serving, {gib} GiB budget: p50 {budgets[-1]['p50_us']} us p99 {budgets[-1]['p99_us']} us, "
            f"{bs['admission_stalls']} admission stalls")

    # per-call FIFO: each job run on arrival with plain plan calls, one at a time;
    # every plan runs one product first, so one-time work (scratch allocation,
    # tables of the split the tuning table picks) stays out of the replay
    plans = {}
    tmp_b = torch.empty(40 << 17, dtype=torch.int64, device="cuda")
    tmp_a = torch.zeros(40 << 17, dtype=torch.int64, device="cuda")
    for j in trace:
        if (j.N, j.L) not in plans:
            p_ = plans[(j.N, j.L)] = ntt.Plan(j.N, primes[:j.L])
            wa = tmp_a[:j.L * j.N].view(j.L, j.N)
            wb = tmp_b[:j.L * j.N].view(j.L, j.N)
            p_.forward(wa, batch=1)
            p_.forward(wb, batch=1)
            p_.pointwise_inverse(wa, wb, wa, batch=1)
    torch.cuda.synchronize()
    fifo_lat = []
    start = time.perf_counter()
    for i, j in enumerate(trace):
        while time.perf_counter() - start < j.arrival_s:
            pass
        op, N, mods, a, out, b = job_args(i, j)
        p_ = plans[(j.N, j.L)]
        o = out[:j.L * j.N].view(j.L, j.N)
        o.copy_(a)
        if op == ntt.NTT_REQ_NTT:
            p_.forward(o, batch=1)
        else:
            bb = tmp_b[:j.L * j.N].view(j.L, j.N)
            bb.copy_(b)
            p_.forward(o, batch=1)
            p_.forward(bb, batch=1)
            p_.pointwise_inverse(o, bb, o, batch=1)
        torch.cuda.synchronize()
        if i >= warm:
            fifo_lat.append((time.perf_counter() - start - j.arrival_s) * 1e6)
    fifo_wall = time.perf_counter() - start
    for p_ in plans.values():
        p_.close()
    fl = np.sort(np.array(fifo_lat))
    res = {"workload": "serving_poisson_ntt_polymul", "jobs": n_jobs, "warmup_jobs": warm,
           "offered_jobs_per_s": round(rate, 1), "saturated_jobs_per_s": round(sat_jobs_s, 1),
           "p50_us": round(st["p50_us"], 1), "p99_us": round(st["p99_us"], 1),
           "ntt_per_s": round(st["ntts"] / st["wall_s"], 1), "batches": st["batches"],
           "mean_jobs_per_batch": round(st["completed"] / max(1, st["batches"]), 2),
           "max_inflight_batches": st["max_inflight_batches"], "admission_stalls": st["admission_stalls"],
           "table_bytes_resident": st["table_bytes"], "table_evictions": st["table_evictions"],
           "hbm_budget_GiB": 4, "load_curve": curve, "budget_sweep_at_70pct": budgets,
           "per_call_fifo": {"p50_us": round(float(fl[len(fl) // 2]), 1),
                             "p99_us": round(float(fl[int(0.99 * (len(fl) - 1))]), 1),
                             "ntt_per_s": round(sum(ntts_of(j) for j in trace) / fifo_wall, 1)}}
    log(f"serving: offered {rate:.0f} jobs/s; server p50 {res['p50_us']} us p99 {res['p99_us']} us; "
        f"per-call FIFO p50 {res['per_call_fifo']['p50_us']} us p99 {res['per_call_fifo']['p99_us']} us")
    return res


POLYMUL_TRACE_KEYS = [("k_col<nttk::Arith64<false, false>, 8, 16, true", "column passes of a and b (one launch)"),
                      ("k_row_polymul<nttk::Arith64<false, false>, 8", "fused rows: both forward, product, first inverse"),
                      ("k_col<nttk::Arith64<false, false>, 8, 16, false", "inverse column pass")]


ROCTX_CMD = ("python3 bench.py --steps 20 --warmup 5 --steady-ms 0 --streams 1 --no-cpu-baseline --no-per-call "
             "--no-batched --no-serving --no-paper-sizes --no-he --no-ablations --no-polymul --no-batch-sweep "
             "--no-latency")


def summarize_roctx(d: str):
    """Writes profiles/roctx_ranges_polymul_n65536_l24.md from a rocprofv3
    marker and kernel trace (rt/*marker_api_trace.csv, rt/*kernel_stats.csv
    under d) of the headline run with NTT_ROCTX=1: the library's ranges per
    call, with their host-side durations, beside the kernels they launched."""
    import csv
    import glob
    ranges = {}
    for f in glob.glob(os.path.join(d, "rt", "*marker_api_trace.csv")):
        for r in csv.DictReader(open(f)):
            msg = r.get("Function") or r.get("Message") or r.get("Name") or ""
            if not msg.startswith("ntt_"):
                continue
            dur = (float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) / 1e3
            ranges.setdefault(msg, []).append(dur)
    stats = {}
    for f in glob.glob(os.path.join(d, "rt", "*kernel_stats.csv")):
        for r in csv.DictReader(open(f)):
            stats[r["Name"]] = r
    lines = ["# roctx ranges: polymul_n65536_l24 (N=2^16, 24 limbs, 2 ciphertexts), MI355X", "",
             "Command (run from the repository root on an MI355X, with the library's ranges switched on):", "",
             "    export NTT_ROCTX=1",
             f"    rocprofv3 --marker-trace --kernel-trace --stats --output-format csv -d <dir>/rt -o rt -- {ROCTX_CMD}",
             "    python3 bench.py --summarize-roctx <dir>", "",
             "Ranges cover the host side of each call (argument checks, variant choice, launches), not the kernels' "
             "execution, which is asynchronous.", "",
             "| range | calls | mean host us | median host us |", "|---|---|---|---|"]
    for name in sorted(ranges):
        v = sorted(ranges[name])
        lines.append(f"| `{name}` | {len(v)} | {sum(v) / len(v):.2f} | {v[len(v) // 2]:.2f} |")
    lines += ["", "| kernel | calls | rocprof avg us |", "|---|---|---|"]
    for name, r in sorted(stats.items(), key=lambda kv: -float(kv[1]["TotalDurationNs"]))[:8]:
        lines.append(f"| `{name.split('(')[0].replace('void ', '')}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} |")
    out = os.path.join(ROOT, "profiles", "roctx_ranges_polymul_n65536_l24.md")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_polymul_trace(d: str):
    """Writes profiles/polymul_fused_n65536_l24_trace.md from the rocprofv3
    kernel trace (kt/*kernel_stats.csv under d) of `bench.py --polymul-only`:
    the three kernels of ntt_polymul at the headline shape, with the per-step
    sum beside the bench's own one-stream step time (bench.json under d)."""
    import csv
    import glob
    stats = {}
    for f in glob.glob(os.path.join(d, "kt", "*kernel_stats.csv")):
        for r in csv.DictReader(open(f)):
            stats[r["Name"]] = r
    cmd = "python3 bench.py --polymul-only --steps 20 --warmup 5 --steady-ms 0"
    lines = ["# Kernel trace: ntt_polymul at polymul_n65536_l24 (N=2^16, 24 limbs, 2 products of 2 components), "
             "MI355X", "",
             "Command (run from the repository root on an MI355X):", "",
             f"    rocprofv3 --kernel-trace --stats --output-format csv -d <dir>/kt -o kt -- {cmd} > <dir>/bench.json",
             f"    python3 bench.py --summarize-polymul-trace <dir>", "",
             f"Kernel source hash: {kernel_source_hash(KERNEL_SOURCES + ['paper_2405_11353_amd/csrc/k_polymul.hip'])}",
             "", "| kernel | role | calls | rocprof avg us |", "|---|---|---|---|"]
    per_step = 0.0
    for pat, role in POLYMUL_TRACE_KEYS:
        rows = [r for n, r in stats.items() if pat in n]
        if not rows:
            continue
        r = rows[0]
        avg = float(r["AverageNs"]) / 1e3
        per_step += avg
        name = r["Name"].split("(")[0].replace("void ", "")
        lines.append(f"| `{name}` | {role} | {r['Calls']} | {avg:.2f} |")
    lines.append("")
    lines.append(f"Sum of the three kernels per step: {per_step:.1f} us.")
    bj = os.path.join(d, "bench.json")
    if os.path.exists(bj):
        res = json.loads(open(bj).read().strip().splitlines()[-1])
        st = res.get("streams_1", {})
        lines.append(f"The same run's `bench.py` step time on one stream (wall clock, launches included): "
                     f"{st.get('us_per_step')} us, {st.get('ntt_equivalent_per_s', 0) / 1e6:.3f} M NTT-equivalent/s.")
    out = os.path.join(ROOT, "profiles", "polymul_fused_n65536_l24_trace.md")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    args = parse()
    if args.summarize_counters:
        summarize_counters(args.summarize_counters)
        return
    if args.summarize_he_counters:
        summarize_counters(args.summarize_he_counters, he=True)
        return
    if args.summarize_polymul_trace:
        summarize_polymul_trace(args.summarize_polymul_trace)
        return
    if args.summarize_roctx:
        summarize_roctx(args.summarize_roctx)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the NTT batch is independent per (polynomial, limb), "
              "so more GPUs would shard limbs with no exchange; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2405_11353_amd as ntt
    import seeded_inputs as si

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)
    if args.he_only:
        clock_warmup(torch, args.clock_warmup_ms)
        print(json.dumps(bench_he_steps(ntt, si, torch)), flush=True)
        return
    if args.polymul_only:
        # one stream, so a kernel trace of this run holds unoverlapped launches
        clock_warmup(torch, args.clock_warmup_ms)
        print(json.dumps(bench_polymul(ntt, si, torch, steps=args.steps, warm=args.warmup, stream_counts=(1,),
                                       steady_ms=args.steady_ms)),
              flush=True)
        return
    w = si.workload_polymul_n16()
    N, moduli, L = w.N, w.moduli, len(w.moduli)
    polys = 4                                       # 2 ciphertexts x 2 components
    set_words = polys * L * N
    set_bytes = set_words * 8
    # a multiple of the stream count, so that steps in flight on different
    # streams never share a buffer set
    n_streams = max(1, args.streams)
    n_sets = math.ceil(max(2, math.ceil((1 << 30) / set_bytes)) / n_streams) * n_streams
    log(f"workload {w.name}: N={N} L={L} polys={polys}; {n_sets} rotating sets of {set_bytes >> 20} MiB")

    host = si.poly_batch(w.seed, polys, moduli, N)  # [4][24][N]: polys 0,1 = ciphertext A, 2,3 = B
    base = torch.from_numpy(host.view(np.int64)).cuda()
    sets = [base.clone() for _ in range(n_sets)]
    plan = ntt.Plan(N, moduli)
    # what the step's calls run with (the tuning table's choice per batch size):
    # the forward on `polys` polynomials, the fused product + inverse on half
    path, logn1 = ntt.ntt_plan_get_variant_for(plan.handle, polys)[:2]
    path_inv, logn1_inv = ntt.ntt_plan_get_variant_for(plan.handle, polys // 2)[:2]
    stream = torch.cuda.current_stream()

    def step(buf, st=None):
        plan.forward(buf, batch=4, stream=st)
        a, b = buf[:2], buf[2:]
        plan.pointwise_inverse(a, b, a, batch=2, stream=st)   # pointwise product fused into the inverse

    # ---- correctness of the timed configuration on one set (vs. an independent
    # GPU check: forward then inverse must return the input exactly)
    chk = base.clone()
    plan.forward(chk, batch=4)
    plan.inverse(chk, batch=4)
    torch.cuda.synchronize()
    assert torch.equal(chk, base), "round trip in the bench configuration is not exact"

    # Consecutive steps alternate between `streams` streams (default priority);
    # each step works on its own buffer set, so a step's inverse passes (48
    # transforms, too few to fill the GPU) overlap the next step's forward
    # passes. With one stream every launch pays its own ramp-up and drain.
    streams = [stream] + [extra_stream(torch, i) for i in range(n_streams - 1)]

    def timed_steps(n_streams):
        sts = streams[:n_streams]
        for s in range(args.warmup):
            step(sets[s % n_sets], sts[s % n_streams])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for st in sts[1:]:
            st.wait_event(e0)
        for s in range(args.steps):
            step(sets[s % n_sets], sts[s % n_streams])
        for st in sts[1:]:
            done = torch.cuda.Event()
            done.record(st)
            stream.wait_event(done)
        e1.record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        return (t1 - t0) * 1e3 / args.steps, e0.elapsed_time(e1) / args.steps

    def steady(n_streams):
        # untimed steps for args.steady_ms before the warm-up steps: from idle,
        # the clocks take tens of milliseconds of sustained load to ramp up, and
        # they drop again within half a second of idling
        sts = streams[:n_streams]
        t0 = time.perf_counter()
        r = 0
        while (time.perf_counter() - t0) * 1e3 < args.steady_ms:
            for _ in range(32):
                step(sets[r % n_sets], sts[r % n_streams])
                r += 1
            torch.cuda.synchronize()

    steady(1)
    ms_wall_1, ms_event_1 = timed_steps(1)
    steady(len(streams))
    ms_wall, ms_event = timed_steps(len(streams)) if len(streams) > 1 else (ms_wall_1, ms_event_1)

    # ---- the timed configuration's output: steps on every stream at once, each
    # on its own buffer set, then each stream's first two components against
    # the oracle on 3 of the 24 limbs (the product of the two ciphertexts)
    import oracle
    chk_sets = [base.clone() for _ in streams]
    torch.cuda.synchronize()
    for st, buf in zip(streams, chk_sets):
        step(buf, st)
    torch.cuda.synchronize()
    limbs = [0, 11, L - 1]
    sub = host[:, limbs]
    spec, _ = oracle.ntt_forward_batch(np.ascontiguousarray(sub), [moduli[l] for l in limbs])
    want, _ = oracle.ntt_inverse_batch(oracle.pointwise_batch(spec[:2], spec[2:], [moduli[l] for l in limbs])[0],
                                       [moduli[l] for l in limbs])
    for buf in chk_sets:
        got = buf.cpu().numpy().view(np.uint64).reshape(host.shape)[:2, limbs]
        assert (got == want).all(), "a timed stream's step differs from the oracle"
    del chk_sets
    log(f"timed configuration checked: {len(streams)} concurrent streams, limbs {limbs} bit-exact vs the oracle")

    # ---- per-step distribution over at least 100 steps (apart from the timed
    # steps above): one stream, events around each step; and with the streams
    # alternating, the intervals between consecutive steps' completions
    n_dist = max(100, args.steps)
    one_dist = dist_us(per_run_us(torch, lambda r: step(sets[r % n_sets], stream), n_dist, stream))
    done_ev = [torch.cuda.Event(enable_timing=True) for _ in range(n_dist + 1)]
    done_ev[0].record(stream)
    for st in streams[1:]:
        st.wait_event(done_ev[0])
    for r in range(n_dist):
        st = streams[r % len(streams)]
        step(sets[r % n_sets], st)
        done_ev[r + 1].record(st)
    torch.cuda.synchronize()
    ends = [done_ev[0].elapsed_time(e) * 1e3 for e in done_ev[1:]]
    ends.sort()
    multi_dist = dist_us([b - a for a, b in zip([0.0] + ends[:-1], ends)])
    log(f"step distribution over {n_dist} steps: one stream mean {one_dist['mean_us']:.1f} p50 {one_dist['p50_us']:.1f} "
        f"p99 {one_dist['p99_us']:.1f} min {one_dist['min_us']:.1f} us; {len(streams)} streams (completion "
        f"intervals) mean {multi_dist['mean_us']:.1f} p50 {multi_dist['p50_us']:.1f} p99 {multi_dist['p99_us']:.1f} us")
    ntts_per_step = polys * L + 2 * L               # 96 forward + 48 inverse
    value = ntts_per_step / (ms_wall / 1e3)
    log(f"step: {ms_wall * 1e3:.1f} us wall, {ms_event * 1e3:.1f} us events on {len(streams)} streams; "
        f"{value / 1e6:.3f} M NTT/s (one stream: {ms_wall_1 * 1e3:.1f} us, "
        f"{ntts_per_step / (ms_wall_1 / 1e3) / 1e6:.3f} M NTT/s)")

    # ---- per-kernel durations with HIP events on the launch stream, after the
    # same clock warm-up as the steps
    clock_warmup(torch, args.clock_warmup_ms)

    def time_kernel(fn, reps):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        for r in range(3):
            fn(sets[r % n_sets])
        torch.cuda.synchronize()
        evs[0].record(stream)
        for r in range(reps):
            fn(sets[r % n_sets])
        evs[1].record(stream)
        torch.cuda.synchronize()
        return evs[0].elapsed_time(evs[1]) / reps * 1e3   # us per launch

    kernels = {}
    # Algorithmic bytes of a transform are 16N (read N words once, write them
    # once), plus each limb's twiddle entries read once per launch (16 B each).
    # The four-step intermediate is not algorithmic: the column pass is credited
    # with the transform's reads, the row pass with its writes (forward), and
    # the fused product + inverse with reading both spectra (its row pass) and
    # writing the product (its column pass). Counter bytes (traffic) beside.
    if path == ntt.NTT_PATH_FOURSTEP and path_inv == ntt.NTT_PATH_FOURSTEP:
        logn2 = int(math.log2(N)) - logn1
        logn2_inv = int(math.log2(N)) - logn1_inv
        twist_fwd, _ = ntt.ntt_plan_get_row_form(plan.handle, polys)
        twist_inv, _ = ntt.ntt_plan_get_row_form(plan.handle, polys // 2)

        def row_table_bytes(twisted, lv, lg1, lg2):
            """Table bytes one launch reads per limb set: the merged row pass all N
            slots; the split-twist pass each row's first-phase twiddles (2^P - 1),
            its NF * TPR twist factors, and the N2 cyclic twiddles."""
            if not twisted:
                return L * 16 * N
            n1, n2 = 1 << lg1, 1 << lg2
            p_ = lg2 % lv or lv
            return L * 16 * (n1 * ((1 << p_) - 1) + n1 * (1 << (lv - p_)) * (n2 >> lv) + n2)

        # column passes read table slots [0, N1) of each limb
        tw_col = L * 16 * (1 << logn1)
        tw_col_inv = L * 16 * (1 << logn1_inv)
        tw_row = row_table_bytes(twist_fwd & ntt.NTT_ROW_TWIST_FWD, 4, logn1, logn2)
        tw_twist = row_table_bytes(twist_inv & ntt.NTT_ROW_TWIST_INV, 3, logn1_inv, logn2_inv)
        kernels["fwd_col_pass"] = dict(fn=lambda b: plan.forward_stage(b, 0, batch=4), items=polys * L,
                                       stages=logn1, extra_muls=0, words_in=1, words_out=0, tw_bytes=tw_col)
        kernels["fwd_row_pass"] = dict(fn=lambda b: plan.forward_stage(b, 1, batch=4), items=polys * L,
                                       stages=logn2, extra_muls=0, words_in=0, words_out=1, tw_bytes=tw_row)
        kernels["inv_row_pass_mul"] = dict(fn=lambda b: plan.pointwise_inverse_stage(b[:2], b[2:], b[:2], 0, batch=2),
                                           items=2 * L, stages=logn2_inv, extra_muls=N, words_in=2, words_out=0,
                                           mont_muls=N, tw_bytes=tw_twist)
        kernels["inv_col_pass"] = dict(fn=lambda b: plan.inverse_stage(b[:2], 1, batch=2), items=2 * L,
                                       stages=logn1_inv, extra_muls=N // 2, words_in=0, words_out=1,
                                       tw_bytes=tw_col_inv)
    else:
        kernels["pointwise"] = dict(fn=lambda b: plan.pointwise(b[:2], b[2:], b[:2], batch=2), items=2 * L,
                                    stages=0, extra_muls=0, words_in=2, words_out=1)
    per_kernel = {}
    for name, k in kernels.items():
        us = time_kernel(k["fn"], args.kernel_reps)
        bytes_alg = k["items"] * N * 8 * (k["words_in"] + k["words_out"]) + k.get("tw_bytes", 0)
        muls = k["items"] * (((N // 2) * k["stages"] + k["extra_muls"]) * MULS_PER_SHOUP
                             + k.get("general_muls", 0) * MULS_PER_GENERAL + k.get("mont_muls", 0) * MULS_PER_MONT)
        gbs = bytes_alg / (us * 1e-6) / 1e9
        tops = muls / (us * 1e-6) / 1e12
        traffic = counter_traffic(name)
        per_kernel[name] = dict(us=round(us, 2), alg_bytes=bytes_alg, alg_int32_muls=muls,
                                hbm_GBs=round(gbs, 1), hbm_frac=round(gbs / HBM_PEAK_GBS, 4),
                                mul_TOPs=round(tops, 3), mul_frac=round(tops / INT32_MUL_PEAK_TOPS, 4),
                                counter_bytes=traffic,
                                counter_over_alg=round(traffic / bytes_alg, 2) if traffic else None)
        log(f"  {name}: {us:.1f} us  {gbs:.0f} GB/s algorithmic ({gbs / HBM_PEAK_GBS:.1%} of HBM peak)  "
            f"{tops:.2f} TOP/s int32 mul ({tops / INT32_MUL_PEAK_TOPS:.1%})")
    # whole transforms: the forward (column + row pass) and the fused product +
    # inverse, each credited 16N (24N with the product) per transform + tables
    transforms = {}
    if path == ntt.NTT_PATH_FOURSTEP:
        for tname, parts in (("forward", ("fwd_col_pass", "fwd_row_pass")),
                             ("product_inverse", ("inv_row_pass_mul", "inv_col_pass"))):
            us = sum(per_kernel[p_]["us"] for p_ in parts)
            b_ = sum(per_kernel[p_]["alg_bytes"] for p_ in parts)
            gbs = b_ / (us * 1e-6) / 1e9
            transforms[tname] = {"us": round(us, 2), "alg_bytes": b_, "hbm_GBs": round(gbs, 1),
                                 "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "kernels": list(parts)}
            log(f"  {tname} transform: {us:.1f} us, {gbs:.0f} GB/s algorithmic ({gbs / HBM_PEAK_GBS:.1%})")
    # the step: 96 forward (16N) + 48 fused product + inverse (24N) + each
    # limb's tables once per direction and pass
    step_bytes = sum(k["alg_bytes"] for k in per_kernel.values())
    step_gbs = step_bytes / (ms_wall * 1e-3) / 1e9
    dominant = max(per_kernel, key=lambda n: per_kernel[n]["us"])
    dk = per_kernel[dominant]
    if dk["mul_frac"] >= dk["hbm_frac"] and dk["alg_int32_muls"] > 0:
        roofline = {"bound": "alu", "achieved": dk["mul_TOPs"], "peak": round(INT32_MUL_PEAK_TOPS, 2),
                    "unit": "TOP/s", "frac": dk["mul_frac"], "traffic": None}
    else:
        roofline = {"bound": "hbm", "achieved": dk["hbm_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": dk["hbm_frac"], "traffic": None}
    roofline["traffic"] = dk["counter_bytes"]
    roofline["traffic_unit"] = "bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a 1 GiB copy)"
    roofline["alg_bytes"] = dk["alg_bytes"]
    roofline["kernel"] = dominant
    roofline["avg_launch_us"] = dk["us"]
    roofline["valu_busy"] = counter_valu_busy(dominant)
    roofline["transforms"] = transforms
    roofline["step"] = {"alg_bytes": step_bytes, "hbm_GBs": round(step_gbs, 1),
                        "hbm_frac": round(step_gbs / HBM_PEAK_GBS, 4), "us": round(ms_wall * 1e3, 2)}
    log(f"roofline: {dominant} at {dk['hbm_frac']:.3f} of 8 TB/s (algorithmic bytes); the step at "
        f"{step_gbs / HBM_PEAK_GBS:.3f}")

    # ---- per-call baseline: the same step as one call per (polynomial, limb)
    per_call = None
    if not args.no_per_call:
        plans = [ntt.Plan(N, [q]) for q in moduli]
        buf = sets[0]

        def step_per_call(bb):
            for p in range(polys):
                for l in range(L):
                    plans[l].forward(bb[p, l], batch=1)
            for p in range(2):
                for l in range(L):
                    plans[l].pointwise(bb[p, l], bb[p + 2, l], bb[p, l], batch=1)
                    plans[l].inverse(bb[p, l], batch=1)

        reps = max(3, args.steps // 20)
        step_per_call(buf)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in range(reps):
            step_per_call(sets[r % n_sets])
        torch.cuda.synchronize()
        ms_pc = (time.perf_counter() - t0) * 1e3 / reps
        per_call = {"ms_per_step": round(ms_pc, 4), "value": round(ntts_per_step / (ms_pc / 1e3), 1),
                    "unit": "NTT/s", "launches_per_step": polys * L * 2 + 2 * L * 3,
                    "batched_speedup": round(ms_pc / ms_wall, 2)}
        log(f"per-call: {ms_pc * 1e3:.1f} us/step, batched speedup {ms_pc / ms_wall:.1f}x")
        for p_ in plans:
            p_.close()

    # ---- CPU oracle on bounded samples of the workloads (and a bit-exact
    # comparison of the GPU's product on the headline sample)
    cpu = None if args.no_cpu_baseline else cpu_baseline(ntt, si, torch, host, base, step,
                                                         seconds=args.cpu_seconds)
    def section(skip, fn, *a, **kw):
        # each GPU section starts from the same clock state (the CPU baseline
        # and the host work between sections leave the GPU idle)
        if skip:
            return None
        clock_warmup(torch, args.clock_warmup_ms)
        return fn(ntt, si, torch, *a, **kw)

    latency = section(args.no_latency, bench_latency)
    batched = section(args.no_batched, bench_batched)
    serving = section(args.no_serving, bench_serving, n_jobs=args.serving_jobs, warm=args.serving_warmup,
                      rate=args.serving_rate)
    paper_sizes = section(args.no_paper_sizes, bench_paper_sizes)
    he_steps = section(args.no_he, bench_he_steps)
    ablations = section(args.no_ablations, bench_ablations)
    polymul = section(args.no_polymul, bench_polymul, steady_ms=args.steady_ms)
    batch_sweep = section(args.no_batch_sweep, bench_batch_sweep)

    res = {
        "metric": "NTT/s at N=2^16 x 24 limbs (forward + inverse NTTs of a batched 2-ciphertext negacyclic product)",
        "value": round(value, 1),
        "unit": "NTT/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_wall, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic: seeded uniform residues mod 24 primes q < 2^60, q = 1 mod 2^17",
        "config": {"workload": w.name, "N": N, "L": L, "polys": polys, "ntts_per_step": ntts_per_step,
                   "variant": {"path": "fourstep" if path == ntt.NTT_PATH_FOURSTEP else "lds", "log_n1": logn1,
                               "log_n1_inverse": logn1_inv},
                   "rotating_sets": n_sets, "footprint_MiB": n_sets * set_bytes >> 20,
                   "streams": len(streams), "untimed_steady_ms": args.steady_ms,
                   "clock_warmup_ms": args.clock_warmup_ms},
        "roofline": roofline,
        "kernels": per_kernel,
        "per_call": per_call,
        "cpu_baseline": cpu,
        "ms_per_step_events": round(ms_event, 5),
        "step_latency": {"one_stream": one_dist, "streams_completion_interval": multi_dist,
                         "streams": len(streams)},
        "latency": latency,
        "one_stream": {"ms_per_step": round(ms_wall_1, 5), "ms_per_step_events": round(ms_event_1, 5),
                       "value": round(ntts_per_step / (ms_wall_1 / 1e3), 1)},
        "batched": batched,
        "serving": serving,
        "paper_sizes": paper_sizes,
        "he_steps": he_steps,
        "ablations": ablations,
        "polymul": polymul,
        "batch_sweep": batch_sweep,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
