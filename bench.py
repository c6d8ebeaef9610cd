"""Throughput benchmark of the batched LDPC decoders on one MI355X.

Default workload: the n = 2304 irregular QC code (Z = 96, 12 x 24 base), offset
min-sum, layered schedule, 20 fixed iterations (no early termination), 65536
codewords per step, BPSK/AWGN at Eb/N0 = 2.0 dB, int8 LLRs.  A step is one
decode of the whole batch with inputs already resident in device memory.

Prints ONE JSON line with the throughput in decoded information bits per
second, a roofline object for the dominant kernel and the CPU oracle timed on
a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue peak: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4 cycles, 2.4 GHz
VALU_PEAK_WAVE_INSTR = 256 * 2.4e9
# Packed 16-bit integer VALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2 halves x 2.4 GHz.
ALU_PEAK_TOPS_I16 = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
PROFILES = os.path.join(ROOT, "profiles")

# Kernel sources whose hash a counter summary is tied to, per kernel family.
FAMILY_SOURCES = {
    "bin_qc_packed": ["k_bin_qc.hip", "dev_bin_qc.h", "dev_common.h"],
    "bin_lds": ["k_bin_lds.hip", "dev_bin_lds.h", "dev_common.h"],
    "bin_interleaved": ["k_bin_il.hip", "dev_bin_il.h", "dev_common.h"],
    "minmax_interleaved": ["k_nb.hip", "dev_nb.h", "dev_common.h"],
    "minmax_lds": ["k_nb.hip", "dev_nb.h", "dev_common.h"],
    "minmax_cw": ["k_nb1.hip", "dev_nb1.h", "dev_common.h"],
    "spa_wave": ["k_spa.hip", "dev_spa.h", "dev_common.h"],
    "spa_lds": ["k_spa.hip", "dev_spa.h", "dev_common.h"],
}


def source_hash(family: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in FAMILY_SOURCES[family] + ["ldpcx_internal.h"]:
        with open(os.path.join(ROOT, "paper_2508_03567_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_counters(workload: str):
    """key: value lines of profiles/<workload>_counters.txt (written from rocprofv3 --pmc runs)."""
    path = os.path.join(PROFILES, f"{workload}_counters.txt")
    if not os.path.exists(path):
        return None
    out = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            out[k.strip()] = v.strip()
    return out


def algorithmic_bytes_per_cw(w) -> float:
    """Bytes the method must move per codeword: compulsory I/O plus, per iteration,
    the compressed message state counted once per datum (flooding: L read n, check
    state read+write 8m, Lambda int16 write+read 4n; layered: 4n + 8m; Min-Max:
    gamma read 2 n g, beta read+write 4 E g)."""
    c = w.code
    n, m, E, g = c.n, c.m, c.nnz, c.g
    if g == 2:
        io = n + (n + 7) // 8 + 1 + 2
        state = 4 * n + 8 * m if w.schedule == "layered" else n + 8 * m + 4 * n
    else:
        io = 2 * n * g + n + 1 + 2
        state = 2 * n * g + 4 * E * g
    return io + w.max_iters * state


# Integer operations of binary min-sum per edge and iteration (one codeword): check node
# (magnitude, minimum and second minimum, sign parity: 6), outgoing message (select,
# normalise, sign: 6), variable node (add, subtract, saturate: 4).
BIN_OPS_PER_EDGE = 16
E2E_WARMUP = 3        # untimed passes of each end-to-end leg, at least ...
E2E_WARMUP_S = 0.08   # ... and at least this long
E2E_SPLIT_BYTES = 16 << 20  # input size from which the overlapped leg runs two chunks (one below:
                             # a small batch decodes faster than the cross-stream waits cost)


def algorithmic_ops_per_cw(w) -> float:
    """Integer operations the method must do per codeword.  Min-Max: per iteration, a max
    and a min for each of the 3 (dc - 2) g^2 pairs of every check (forward, backward and
    middle-beta convolutions) plus about 6 E g for the variable nodes.  Binary min-sum:
    BIN_OPS_PER_EDGE per edge and iteration."""
    c = w.code
    if c.g == 2:
        return float(w.max_iters) * BIN_OPS_PER_EDGE * c.nnz
    dc = np.diff(np.asarray(c.row_ptr))
    cn = float(np.sum(2 * 3 * np.maximum(dc - 2, 0))) * c.g * c.g
    return w.max_iters * (cn + 6.0 * c.nnz * c.g)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=1, help="0..3: n192 NMS, n2304 OMS layered, n64800 NMS, GF(64)")
    ap.add_argument("--batch", type=int, default=None)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--plan", type=str, default=None,
                    help="pin the launch plan instead of tuning: family[:cw_per_wg[:threads]], e.g. bin_interleaved:256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-e2e", action="store_true", help="skip the end-to-end (PCIe-inclusive) leg")
    ap.add_argument("--e2e-chunks", type=int, default=0,
                    help="chunks of the overlapped end-to-end leg (0: 2 from 16 MiB of input up, else 1)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU oracle time")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after timing, run one 256 MiB device-to-device copy (counter calibration)")
    ap.add_argument("--serve", action="store_true",
                    help="serving mix instead: Poisson arrivals of mixed requests, continuous batching vs "
                         "per-request decoding, p50/p99 latency (one JSON line per mode and load)")
    ap.add_argument("--rho", type=str, default="0.1,0.3,0.5,0.7,0.9,1.1", help="--serve: loads, fractions of capacity")
    ap.add_argument("--requests", type=int, default=2000, help="--serve: measured requests per load")
    ap.add_argument("--warm-requests", type=int, default=200, help="--serve: warm-up requests per load")
    ap.add_argument("--budget-gib", type=float, default=8.0, help="--serve: server HBM budget")
    ap.add_argument("--modes", type=str, default="continuous,per_request", help="--serve: serving modes")
    ap.add_argument("--precision", action="store_true",
                    help="Min-Max message precision: 16-bit vs 8-bit (bound 127) messages on the GF(64) workload, "
                         "FER over Eb/N0 and fixed-iteration throughput")
    ap.add_argument("--ebn0-sweep", action="store_true",
                    help="headline code over its Eb/N0 sweep (1.0-3.0 dB): FER, mean iterations and throughput "
                         "with syndrome early stop, and at fixed iterations")
    ap.add_argument("--peaks", action="store_true",
                    help="measured device peaks: copy bandwidth over buffer sizes and the packed 16-bit VALU "
                         "issue rate, against the spec figures")
    ap.add_argument("--ragged", action="store_true",
                    help="ragged batch of small mixed jobs: one persistent launch vs one decode call per job")
    ap.add_argument("--schedule", type=str, default=None, choices=["flooding", "layered"],
                    help="override the workload's schedule (the workload name then carries it)")
    ap.add_argument("--schedules", action="store_true",
                    help="Min-Max flooding vs layered on the GF(64) workload: FER at fixed iteration counts, "
                         "mean iterations and time with early stop, fixed-iteration throughput")
    ap.add_argument("--sweep", action="store_true",
                    help="GF-size sweep instead: (2,4)-regular codes of 16/32/64 symbols over GF(4)..GF(256), "
                         "Min-Max, fixed iterations (one JSON line per point)")
    ap.add_argument("--sweep-rule", type=str, default="minmax", choices=["minmax", "spa"],
                    help="--sweep: decoder")
    ap.add_argument("--sweep-fields", type=str, default=None, help="--sweep: comma-separated field sizes (default all)")
    ap.add_argument("--prof-summary", type=str, default=None,
                    help="summarise rocprofv3 CSV output instead of running: comma-separated output directories "
                         "(one kernel-trace run, or the --pmc runs of one counter summary)")
    ap.add_argument("--prof-kernel", type=str, default=None,
                    help="--prof-summary: substring naming the decoder kernels (default: all kernels but copies)")
    ap.add_argument("--prof-skip", type=int, default=0,
                    help="--prof-summary: decodes at the start to leave out (warm-up)")
    ap.add_argument("--prof-decodes", type=int, default=1, help="--prof-summary: decodes that follow them")
    ap.add_argument("--prof-family", type=str, default=None,
                    help="--prof-summary of counters: kernel family whose source hash the summary carries")
    ap.add_argument("--prof-title", type=str, default="", help="--prof-summary: workload name for the heading")
    ap.add_argument("--prof-cmd", type=str, default="", help="--prof-summary: command(s) that made the output")
    args = ap.parse_args()

    if args.prof_summary:
        prof_main(args)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); codewords are "
              "independent, so a multi-GPU run would split the batch with no exchange step.", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        serve_main(args)
        return
    if args.sweep:
        sweep_main(args)
        return
    if args.precision:
        precision_main(args)
        return
    if args.schedules:
        schedules_main(args)
        return
    if args.ragged:
        ragged_main(args)
        return
    if args.peaks:
        peaks_main(args)
        return
    if args.ebn0_sweep:
        ebn0_main(args)
        return

    import torch
    from paper_2508_03567_amd import ldpcx as L
    from paper_2508_03567_amd import synth as S

    w = S.workload(args.workload, batch=args.batch)
    if args.schedule and args.schedule != w.schedule:
        import dataclasses
        w = dataclasses.replace(w, schedule=args.schedule, name=f"{w.name}_{args.schedule}")
    t0 = time.time()
    cw, llr_np = S.make_inputs(w)
    gen_s = time.time() - t0
    print(f"bench: workload {w.name} batch {w.batch} inputs generated in {gen_s:.1f}s", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    llr = torch.from_numpy(llr_np).to(dev)
    code = L.Code(w.code)
    prm = L.params(w.rule, w.schedule, w.max_iters, early_stop=False, nms_num=w.nms_num, nms_shift=w.nms_shift,
                   oms_offset=w.oms_offset, msg_max=w.msg_max)
    if args.plan:
        parts = args.plan.split(":")
        L.plan_set(code, prm, w.batch, parts[0], *[int(x) for x in parts[1:]])
    elif not args.no_tune:
        sched, us = L.tune(code, prm, w.batch)
        print(f"bench: tuned plan {L.plan_info(code, prm, w.batch)} ({us:.0f} us)", file=sys.stderr, flush=True)
    plan = L.plan_info(code, prm, w.batch)
    out = L._outputs(code, w.batch, dev)
    for _ in range(args.warmup):
        L.decode(code, prm, llr, out=out)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        L.decode(code, prm, llr, stream=stream, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)

    info_bits = w.info_bits_per_cw * w.batch * args.steps
    value = info_bits / wall / 1e9
    ms_per_step = wall * 1e3 / args.steps
    # The plain decode is one kernel launch for the LDS-resident family; for the
    # interleaved families the event window covers the whole per-iteration sequence.
    kernel_ms = ev_ms / args.steps
    alg_bytes = algorithmic_bytes_per_cw(w) * w.batch
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9

    # End to end, PCIe included: pinned host LLRs in, decisions, flags and iteration
    # counts back to pinned host memory, on the same stream.
    e2e = None
    e2e_steps = 0 if args.no_e2e else max(1, min(args.steps, 5))
    llr_host = torch.from_numpy(llr_np).pin_memory()
    host_out = [torch.empty(o.shape, dtype=o.dtype, pin_memory=True) for o in out]
    llr_dev = torch.empty_like(llr)
    # The first passes over pinned host buffers block the host in the copy calls for
    # milliseconds (for some tens of milliseconds after the buffers are first used); both
    # end-to-end legs are timed after untimed passes.

    def warm(fn):
        t_w, k = time.perf_counter(), 0
        while k < E2E_WARMUP or time.perf_counter() - t_w < E2E_WARMUP_S:
            fn()
            torch.cuda.synchronize()
            k += 1

    def serial():
        llr_dev.copy_(llr_host, non_blocking=True)
        L.decode(code, prm, llr_dev, stream=stream, out=out)
        for ho, o in zip(host_out, out):
            ho.copy_(o, non_blocking=True)

    if e2e_steps:
        warm(serial)
    t1 = time.perf_counter()
    for _ in range(e2e_steps):
        serial()
    torch.cuda.synchronize()
    if e2e_steps:
        e2e_ms = (time.perf_counter() - t1) * 1e3 / e2e_steps
        e2e = {"info_gbit_s": round(w.info_bits_per_cw * w.batch / (e2e_ms * 1e-3) / 1e9, 4),
               "ms_per_batch": round(e2e_ms, 4), "steps": e2e_steps,
               "what": "pinned host LLRs -> device, decode, outputs -> pinned host"}
        # The same in chunks on three streams (inputs in, decode, outputs out), chained by
        # per-chunk events: the input copies run back to back while earlier chunks decode,
        # and each chunk's outputs go back while later chunks decode.  A chunk's device
        # buffers are reused by the next pass only after its decode / output copy of this
        # pass has finished, so consecutive passes overlap too (the rate is that of a
        # continuous stream of batches).  The events are created once and re-recorded
        # every pass.
        in_bytes = llr_host.numel() * llr_host.element_size()
        nch = args.e2e_chunks if args.e2e_chunks > 0 else (2 if in_bytes >= E2E_SPLIT_BYTES else 1)
        step_cw = (w.batch + nch - 1) // nch
        chunks = [(c0, min(w.batch, c0 + step_cw)) for c0 in range(0, w.batch, step_cw)]
        s_in, s_dec, s_out = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
        outs = [[o[a:b] for o in out] for a, b in chunks]
        hosts = [[ho[a:b] for ho in host_out] for a, b in chunks]
        ev_in, ev_dec, ev_out = ([torch.cuda.Event() for _ in chunks] for _ in range(3))
        passes = [0]

        def pipelined():
            later = passes[0] > 0  # the previous pass's decode / output copy of a chunk is pending
            for i, (a, b) in enumerate(chunks):
                if later:
                    s_in.wait_event(ev_dec[i])
                with torch.cuda.stream(s_in):
                    llr_dev[a:b].copy_(llr_host[a:b], non_blocking=True)
                ev_in[i].record(s_in)
            for i, (a, b) in enumerate(chunks):
                s_dec.wait_event(ev_in[i])
                if later:
                    s_dec.wait_event(ev_out[i])
                L.decode(code, prm, llr_dev[a:b], stream=s_dec, out=outs[i])
                ev_dec[i].record(s_dec)
            for i in range(len(chunks)):
                s_out.wait_event(ev_dec[i])
                with torch.cuda.stream(s_out):
                    for ho, o in zip(hosts[i], outs[i]):
                        ho.copy_(o, non_blocking=True)
                ev_out[i].record(s_out)
            passes[0] += 1

        warm(pipelined)
        t2 = time.perf_counter()
        for _ in range(e2e_steps):
            pipelined()
        torch.cuda.synchronize()
        ov_ms = (time.perf_counter() - t2) * 1e3 / e2e_steps
        e2e["overlapped_info_gbit_s"] = round(w.info_bits_per_cw * w.batch / (ov_ms * 1e-3) / 1e9, 4)
        e2e["overlapped_ms_per_batch"] = round(ov_ms, 4)
        e2e["overlapped_what"] = (f"{len(chunks)} chunks on three streams (inputs in, decode, outputs out), "
                                  "passes back to back: copies of one chunk overlap the decode of others")

    if args.calib_copy:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()

    traffic, valu_frac = None, None
    ctr = read_counters(w.name)
    if ctr and ctr.get("source_hash") == source_hash(plan["family"]) and ctr.get("family") == plan["family"]:
        traffic = float(ctr["hbm_bytes_per_launch"])
        if "valu_wave_instr_per_launch" in ctr:
            valu_frac = float(ctr["valu_wave_instr_per_launch"]) / (kernel_ms * 1e-3) / VALU_PEAK_WAVE_INSTR

    hard, ok, it = out
    torch.cuda.synchronize()
    h = hard.cpu().numpy()
    if w.code.g == 2:
        h = L.unpack_bits(h, w.code.n)
    fer = float((h != cw).any(axis=1).mean())

    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        nthreads = len(os.sched_getaffinity(0))
        prm_o = O.params(w.rule, w.schedule, w.max_iters, False, w.nms_num, w.nms_shift, w.oms_offset, w.msg_max)
        dec = O.decode_binary if w.code.g == 2 else O.decode_nb
        # Calibrate on a growing sample, then time passes over a sample sized for about
        # cpu_seconds (whole passes over the batch when the batch is faster than that).
        k, per_cw = min(w.batch, 4 * nthreads), None
        while True:
            t1 = time.perf_counter()
            dec(w.code, prm_o, llr_np[:k], nthreads=nthreads)
            dt = time.perf_counter() - t1
            per_cw = dt / k
            if dt > 0.5 or k == w.batch:
                break
            k = min(w.batch, k * 8)
        k = int(min(w.batch, max(4 * nthreads, args.cpu_seconds / max(per_cw, 1e-9))))
        done_cw, cpu_s, passes = 0, 0.0, 0
        while cpu_s < args.cpu_seconds and passes < 100000:
            t1 = time.perf_counter()
            dec(w.code, prm_o, llr_np[:k], nthreads=nthreads)
            cpu_s += time.perf_counter() - t1
            done_cw += k
            passes += 1
        cpu = {"value": round(done_cw * w.info_bits_per_cw / cpu_s / 1e9, 6), "unit": "Gbit/s", "cores": nthreads,
               "kind": "oracle",
               "sample": f"{passes} pass(es) over the first {k} of the {w.batch} codewords, "
                         f"{w.max_iters} fixed iterations, {cpu_s:.1f}s",
               "cpu_model": cpu_model()}
        # One core: the same oracle, passes over a sample until about a quarter of that time.
        k1 = int(min(w.batch, max(1, 0.25 * args.cpu_seconds / max(per_cw * nthreads, 1e-9))))
        s1, p1 = 0.0, 0
        while s1 < 0.25 * args.cpu_seconds and p1 < 100000:
            t1 = time.perf_counter()
            dec(w.code, prm_o, llr_np[:k1], nthreads=1)
            s1 += time.perf_counter() - t1
            p1 += 1
        cpu["one_core"] = {"value": round(p1 * k1 * w.info_bits_per_cw / s1 / 1e9, 6), "unit": "Gbit/s",
                           "sample": f"{p1} pass(es) over the first {k1} codewords, {w.max_iters} fixed iterations, "
                                     f"{s1:.1f}s"}

    alg_ops = algorithmic_ops_per_cw(w) * w.batch
    tops = alg_ops / (kernel_ms * 1e-3) / 1e12
    if plan["family"] == "bin_interleaved":
        # message state streams through device memory every iteration: bound by HBM
        roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "alu_achieved_tops": round(tops, 3),
                "alu_frac": round(tops / ALU_PEAK_TOPS_I16, 4)}
    else:
        # The on-chip binary families (device memory carries only the I/O) and Min-Max are
        # bound by packed 16-bit integer VALU work; the modelled state bytes per second
        # are kept beside it as an effective bandwidth, not a roof this kernel meets.
        roof = {"bound": "alu", "achieved": round(tops, 3), "peak": round(ALU_PEAK_TOPS_I16, 2), "unit": "Tops/s int16",
                "frac": round(tops / ALU_PEAK_TOPS_I16, 4),
                "hbm_model_gbs": round(achieved, 2), "hbm_model_frac": round(achieved / HBM_PEAK_GBS, 4)}
    roof.update({"traffic": traffic, "hbm_measured_gbs": None if traffic is None else
                 round(traffic / (kernel_ms * 1e-3) / 1e9, 2),
                 "valu_frac": None if valu_frac is None else round(valu_frac, 4),
                 "kernel_ms": round(kernel_ms, 4), "algorithmic_ops_per_launch": int(alg_ops),
                 "algorithmic_bytes_per_launch": int(alg_bytes)})
    res = {
        "metric": "decoded info Gbit/s at fixed iters",
        "value": round(value, 4),
        "unit": "Gbit/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8" if w.code.g == 2 else "int16",
        "data": "synthetic: seeded random info bits, encoded, BPSK over AWGN, quantised LLRs",
        "config": {"workload": w.name, "n": w.code.n, "k_info": w.code.k_info, "field": w.code.g,
                   "rule": w.rule, "schedule": w.schedule, "iterations": w.max_iters, "early_stop": False,
                   "batch": w.batch, "ebn0_db": w.ebn0_db, "plan": plan,
                   "coded_gbit_s": round(value * w.code.n / w.code.k_info, 4), "fer": fer},
        "roofline": roof,
        "end_to_end": e2e,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


# ------------------------------------------------------------------ rocprofv3 summaries
def _prof_rows(dirs, suffix):
    """Rows of every rocprofv3 CSV whose name ends in `suffix` under the directories."""
    import csv
    rows = []
    for d in dirs:
        for root, _, files in os.walk(d):
            for f in sorted(files):
                if f.endswith(suffix):
                    with open(os.path.join(root, f), newline="") as fh:
                        rows.extend(csv.DictReader(fh))
    return rows


def _is_copy(name: str) -> bool:
    return "copyBuffer" in name or "fillBuffer" in name or "FillFunctor" in name or "elementwise" in name


def prof_main(args) -> None:
    """Summaries of rocprofv3 runs of this benchmark for profiles/.

    Kernel trace: per kernel, calls and mean / median / min / max duration over the whole
    run, then the decoder kernels of the timed decodes only (the first --prof-skip decodes'
    dispatches left out), summed per decode.  Counters (--pmc runs): the decoder kernels'
    counters summed over the timed decodes' dispatches and divided by --prof-decodes, with
    FETCH_SIZE and WRITE_SIZE scaled by what they read for the 256 MiB device copy that
    --calib-copy runs at the end."""
    dirs = [d for d in args.prof_summary.split(",") if d]
    sel = (lambda nm: args.prof_kernel in nm) if args.prof_kernel else (lambda nm: not _is_copy(nm))
    trace = _prof_rows(dirs, "kernel_trace.csv")
    ctr = _prof_rows(dirs, "counter_collection.csv")
    K, W = max(1, args.prof_decodes), max(0, args.prof_skip)
    if trace and not ctr:
        by = {}
        order = []
        for r in trace:
            nm = r["Kernel_Name"]
            dt = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            if nm not in by:
                by[nm] = []
                order.append(nm)
            by[nm].append((int(r["Start_Timestamp"]), dt))
        total = sum(dt for v in by.values() for _, dt in v)
        print(f"# rocprofv3 kernel statistics: {args.prof_title}\n")
        print(f"Command (rocprofv3 writes its CSV files to the -d directory):\n\n```\n{args.prof_cmd}\n```\n")
        print("| kernel | calls | mean ns | median ns | min ns | max ns | % of GPU time |")
        print("|---|---|---|---|---|---|---|")
        for nm in sorted(order, key=lambda n: -sum(dt for _, dt in by[n])):
            d = np.array([dt for _, dt in by[nm]], dtype=np.float64)
            print(f"| `{nm[:110]}` | {len(d)} | {d.mean():.0f} | {np.median(d):.0f} | {d.min():.0f} | {d.max():.0f} "
                  f"| {100 * d.sum() / total:.2f} |")
        if not args.prof_kernel:
            return
        dec = sorted((t, dt) for nm in order if sel(nm) for t, dt in by[nm])
        n_all = len(dec)
        per = n_all // (W + K) if n_all % (W + K) == 0 else None
        if per is None:
            print(f"\n{n_all} decoder dispatches do not split evenly into {W} + {K} decodes.")
            return
        timed = np.array([dt for _, dt in dec[W * per:]], dtype=np.float64).reshape(K, per).sum(axis=1)
        print(f"\nDecoder kernels: {per} dispatch(es) per decode; {W} warm-up decode(s) left out; over the "
              f"{K} timed decodes the kernel time per decode is mean {timed.mean():.0f} ns, median "
              f"{np.median(timed):.0f} ns, min {timed.min():.0f} ns, max {timed.max():.0f} ns.")
        return
    if not ctr:
        print("no rocprofv3 CSV output found under " + ", ".join(dirs), file=sys.stderr)
        sys.exit(1)
    # counters: dispatch -> {counter: value}
    disp = {}
    for r in ctr:
        key = (r.get("Process_Id", ""), r["Dispatch_Id"])
        e = disp.setdefault(key, {"name": r["Kernel_Name"], "t": int(r.get("Start_Timestamp", 0) or 0), "c": {}})
        e["c"][r["Counter_Name"]] = e["c"].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    names = sorted({c for e in disp.values() for c in e["c"]})
    out = {}
    for cname in names:
        rows = sorted((e["t"], e) for e in disp.values() if cname in e["c"])
        dec = [e for _, e in rows if sel(e["name"])]
        per = len(dec) // (W + K) if len(dec) % (W + K) == 0 else None
        if not per:
            print(f"{cname}: {len(dec)} decoder dispatches do not split into {W} + {K} decodes", file=sys.stderr)
            sys.exit(1)
        out[cname] = sum(e["c"][cname] for e in dec[W * per:]) / K
        out[cname + "_dispatches"] = per
        copies = [e["c"][cname] for _, e in rows if "copyBuffer" in e["name"]]
        if cname in ("FETCH_SIZE", "WRITE_SIZE") and copies:
            out[cname + "_scale"] = 262144.0 / max(copies)
    print(f"# HBM traffic and VALU instruction counters per decode, workload {args.prof_title}")
    for line in args.prof_cmd.split(";;"):
        print(f"# run: {line.strip()}")
    print("# Counters are summed over the decoder kernels of the timed decodes (warm-up left out).")
    print("# FETCH_SIZE and WRITE_SIZE (KiB) are scaled by 256 MiB over what they read for the 256 MiB")
    print("# device-to-device copy run at the end of the same command.")
    if args.prof_family:
        print(f"family: {args.prof_family}")
        print(f"source_hash: {source_hash(args.prof_family)}")
    print(f"decodes: {K}")
    hbm = 0.0
    for cname in ("FETCH_SIZE", "WRITE_SIZE"):
        if cname in out:
            sc = out.get(cname + "_scale", 1.0)
            print(f"{cname.lower()}_kib_per_launch_raw: {out[cname]:.1f}")
            print(f"{cname.lower()}_scale: {sc:.4f}")
            hbm += out[cname] * sc * 1024
    if "FETCH_SIZE" in out and "WRITE_SIZE" in out:
        print(f"hbm_bytes_per_launch: {hbm:.0f}")
    if "SQ_INSTS_VALU" in out:
        print(f"valu_wave_instr_per_launch: {out['SQ_INSTS_VALU']:.0f}")
    if "SQ_WAVES" in out:
        print(f"waves_per_launch: {out['SQ_WAVES']:.0f}")
    for cname in names:
        if cname not in ("FETCH_SIZE", "WRITE_SIZE", "SQ_INSTS_VALU", "SQ_WAVES"):
            print(f"{cname.lower()}_per_launch: {out[cname]:.0f}")


# ------------------------------------------------------------------ GF-size sweep
SWEEP_N = (16, 32, 64)
SWEEP_G = (4, 8, 16, 32, 64, 128, 256)


def sweep_main(args) -> None:
    """Throughput of the Min-Max decoders over field size and code length, on seeded
    (2,4)-regular codes shaped like the paper's C1-C3 (16, 32, 64 symbols, rate 1/2)."""
    import torch
    from paper_2508_03567_amd import ldpcx as L
    from paper_2508_03567_amd import synth as S

    dev = torch.device("cuda:0")
    iters = 20
    rule = args.sweep_rule
    for n in SWEEP_N:
        for g in SWEEP_G:
            if args.sweep_fields and g not in [int(x) for x in args.sweep_fields.split(",")]:
                continue
            batch = args.batch or 8192
            code = S.random_regular_nb_code(n, n // 2, 2, 4, g, S.PRIM_POLY[g], seed=100 + n + g, name=f"n{n}_gf{g}")
            cw = S.random_codewords(code, batch, seed=7)
            gam = torch.from_numpy(S.nb_gamma_int16(cw, g, 2.0, seed=8)).to(dev)
            h = L.Code(code)
            prm = L.params(rule, "flooding", iters, early_stop=False)
            if not args.no_tune:
                L.tune(h, prm, batch)
            plan = L.plan_info(h, prm, batch)
            out = L._outputs(h, batch, dev)
            for _ in range(max(1, args.warmup)):
                L.decode(h, prm, gam, out=out)
            torch.cuda.synchronize()
            stream = torch.cuda.current_stream()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            steps = max(1, min(args.steps, 5))
            ev0.record(stream)
            for _ in range(steps):
                L.decode(h, prm, gam, stream=stream, out=out)
            ev1.record(stream)
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1) / steps
            p = g.bit_length() - 1
            info = (n // 2) * p * batch / (ms * 1e-3) / 1e9
            fer = float((out[0].cpu().numpy() != cw).any(axis=1).mean())
            print(json.dumps({"metric": f"{rule} GF-size sweep: decoded info Gbit/s at fixed iters", "plan": plan,
                              "n_symbols": n,
                              "field": g, "iterations": iters, "batch": batch, "ms_per_batch": round(ms, 4),
                              "info_gbit_s": round(info, 5), "coded_gbit_s": round(2 * info, 5),
                              "ebn0_db": 2.0, "fer": fer, "data": "synthetic seeded BPSK/AWGN"}), flush=True)
            del gam, out, h
            torch.cuda.empty_cache()


def precision_main(args) -> None:
    """FER and throughput of the GF(64) Min-Max decoder with 16-bit and 8-bit messages."""
    import torch
    from paper_2508_03567_amd import ldpcx as L
    from paper_2508_03567_amd import synth as S

    dev = torch.device("cuda:0")
    for eb in (1.5, 2.0, 2.5, 3.0):
        w = S.workload(3, batch=args.batch or 8192, ebn0_db=eb)
        cw, gam_np = S.make_inputs(w)
        gam = torch.from_numpy(gam_np).to(dev)
        h = L.Code(w.code)
        for bound, name in ((0, "int16"), (127, "int8")):
            prm = L.params("minmax", "flooding", w.max_iters, early_stop=True, nb_msg_max=bound)
            hard, ok, it, _ = L.decode(h, prm, gam)
            torch.cuda.synchronize()
            fer = float((hard.cpu().numpy() != cw).any(axis=1).mean())
            mean_it = float(it.float().mean())
            prm_fixed = L.params("minmax", "flooding", w.max_iters, early_stop=False, nb_msg_max=bound)
            out = L._outputs(h, w.batch, dev)
            L.decode(h, prm_fixed, gam, out=out)
            torch.cuda.synchronize()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            stream = torch.cuda.current_stream()
            ev0.record(stream)
            for _ in range(3):
                L.decode(h, prm_fixed, gam, stream=stream, out=out)
            ev1.record(stream)
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1) / 3
            # The one-codeword-per-workgroup family stores the messages in the width the
            # bound needs (8 bits for 127): the storage half of the precision comparison.
            ms_cw = None
            if eb == 2.0:
                L.plan_set(h, prm_fixed, w.batch, "minmax_cw", 1, 512)
                L.decode(h, prm_fixed, gam, out=out)
                torch.cuda.synchronize()
                ev0.record(stream)
                for _ in range(3):
                    L.decode(h, prm_fixed, gam, stream=stream, out=out)
                ev1.record(stream)
                torch.cuda.synchronize()
                ms_cw = ev0.elapsed_time(ev1) / 3
                h = L.Code(w.code)  # drop the pinned plan
            print(json.dumps({"metric": "Min-Max message precision", "messages": name, "ebn0_db": eb, "fer": fer,
                              "mean_iters": round(mean_it, 3), "workload": w.name, "batch": w.batch,
                              "fixed_iter_info_gbit_s": round(w.info_bits_per_cw * w.batch / (ms * 1e-3) / 1e9, 4),
                              "fixed_iter_info_gbit_s_one_cw_family": None if ms_cw is None else
                              round(w.info_bits_per_cw * w.batch / (ms_cw * 1e-3) / 1e9, 4),
                              "storage_bits_one_cw_family": 8 if bound and bound <= 255 else 16}),
                  flush=True)


def _time_decode(L, torch, h, prm, gam, out, reps=3):
    stream = torch.cuda.current_stream()
    L.decode(h, prm, gam, stream=stream, out=out)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        L.decode(h, prm, gam, stream=stream, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / reps


def schedules_main(args) -> None:
    """Min-Max with the two-phase (flooding) and the layered schedule on the GF(64) workload."""
    import torch
    from paper_2508_03567_amd import ldpcx as L
    from paper_2508_03567_amd import synth as S

    dev = torch.device("cuda:0")
    for eb in (1.5, 2.0, 2.5):
        w = S.workload(3, batch=args.batch or 8192, ebn0_db=eb)
        cw, gam_np = S.make_inputs(w)
        gam = torch.from_numpy(gam_np).to(dev)
        h = L.Code(w.code)
        out = L._outputs(h, w.batch, dev)
        for sched in ("flooding", "layered"):
            rec = {"metric": "Min-Max schedule", "schedule": sched, "ebn0_db": eb, "workload": w.name,
                   "batch": w.batch}
            for iters in (5, 10, 20):
                hard, ok, it, _ = L.decode(h, L.params("minmax", sched, iters, early_stop=False), gam, out=out)
                torch.cuda.synchronize()
                rec[f"fer_{iters}it"] = float((hard.cpu().numpy() != cw).any(axis=1).mean())
            prm_es = L.params("minmax", sched, w.max_iters, early_stop=True)
            hard, ok, it, _ = L.decode(h, prm_es, gam, out=out)
            torch.cuda.synchronize()
            rec["mean_iters_early_stop"] = round(float(it.float().mean()), 3)
            ms_es = _time_decode(L, torch, h, prm_es, gam, out)
            ms_fx = _time_decode(L, torch, h, L.params("minmax", sched, w.max_iters, early_stop=False), gam, out)
            rec["ms_early_stop"] = round(ms_es, 3)
            rec["info_gbit_s_early_stop"] = round(w.info_bits_per_cw * w.batch / (ms_es * 1e-3) / 1e9, 4)
            rec["ms_fixed_20it"] = round(ms_fx, 3)
            rec["info_gbit_s_fixed_20it"] = round(w.info_bits_per_cw * w.batch / (ms_fx * 1e-3) / 1e9, 4)
            print(json.dumps(rec), flush=True)


def ebn0_main(args) -> None:
    """The headline n = 2304 QC code (OMS, layered, I_max = 20, 65536 codewords) over its
    Eb/N0 sweep: with syndrome early stop (FER, mean iterations, throughput) and at fixed
    iterations."""
    import torch
    from paper_2508_03567_amd import ldpcx as L
    from paper_2508_03567_amd import synth as S

    dev = torch.device("cuda:0")
    for eb in (1.0, 1.5, 2.0, 2.5, 3.0):
        w = S.workload(1, batch=args.batch, ebn0_db=eb)
        cw, llr_np = S.make_inputs(w)
        llr = torch.from_numpy(llr_np).to(dev)
        h = L.Code(w.code)
        out = L._outputs(h, w.batch, dev)
        rec = {"metric": "headline code over Eb/N0", "workload": w.name, "ebn0_db": eb, "batch": w.batch}
        for es in (True, False):
            prm = L.params(w.rule, w.schedule, w.max_iters, early_stop=es, nms_num=w.nms_num, nms_shift=w.nms_shift,
                           oms_offset=w.oms_offset, msg_max=w.msg_max)
            L.tune(h, prm, w.batch)
            ms = _time_decode(L, torch, h, prm, llr, out, reps=5)
            key = "early_stop" if es else "fixed_20it"
            rec[f"info_gbit_s_{key}"] = round(w.info_bits_per_cw * w.batch / (ms * 1e-3) / 1e9, 3)
            rec[f"ms_{key}"] = round(ms, 3)
            if es:
                hard, ok, it = out
                torch.cuda.synchronize()
                h_np = L.unpack_bits(hard.cpu().numpy(), w.code.n)
                rec["fer"] = float((h_np != cw).any(axis=1).mean())
                rec["mean_iters"] = round(float(it.float().mean()), 3)
        print(json.dumps(rec), flush=True)


def peaks_main(args) -> None:
    """Measured peaks of this GPU next to the spec ones: device-to-device copy rate
    (read + write bytes) over buffer sizes, and the packed 16-bit VALU issue rate."""
    import torch
    from paper_2508_03567_amd import ldpcx as L

    dev = torch.device("cuda:0")
    for mb in (16, 64, 128, 256, 512, 2048):
        n = mb * 1024 * 1024 // 4
        src = torch.ones(n, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        reps = max(5, 4096 // mb)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        print(json.dumps({"metric": "device copy rate (read + write bytes)", "buffer_mb": mb,
                          "tb_s": round(2 * mb * 2 ** 20 / (ms * 1e-3) / 1e12, 3), "spec_tb_s": HBM_PEAK_GBS / 1e3}),
              flush=True)
        del src, dst
    stream = torch.cuda.current_stream()
    blocks, iters = 256 * 8 * 4, 4096
    L.valu_probe(blocks, 64, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    L.valu_probe(blocks, iters, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    wave_instr = blocks * 4 * iters * 16
    rate = wave_instr / (ms * 1e-3)
    print(json.dumps({"metric": "packed 16-bit VALU issue rate", "wave_instr_per_s": round(rate / 1e9, 2),
                      "int16_tops": round(rate * 128 / 1e12, 2), "spec_wave_instr_per_s": VALU_PEAK_WAVE_INSTR / 1e9,
                      "spec_int16_tops": round(ALU_PEAK_TOPS_I16, 2), "frac_of_spec": round(rate / VALU_PEAK_WAVE_INSTR, 4),
                      "ms": round(ms, 3)}), flush=True)


def ragged_main(args) -> None:
    """Many small jobs of the three short codes (n = 192 binary, n = 2304 binary, GF(64)),
    1 to 256 codewords each (log-uniform), early stop on: one ldpcx_decode_ragged launch
    against a loop of ldpcx_decode calls, one per job, on the same stream."""
    # Plain per-job decodes run their launch sequences eagerly: graph replays are keyed by
    # the I/O buffers and would be captured anew for every job slice.
    os.environ["LDPCX_GRAPHS"] = "0"
    import torch
    from paper_2508_03567_amd import ldpcx as L
    from paper_2508_03567_amd import synth as S

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(31)
    pools, codes, prms = {}, {}, {}
    for cfg in (0, 1, 3):
        w = S.workload(cfg, batch=512)
        _, llr = S.make_inputs(w, seed_offset=310)
        pools[cfg] = torch.from_numpy(np.ascontiguousarray(llr)).to(dev)
        codes[cfg] = L.Code(w.code)
        prms[cfg] = L.params(w.rule, w.schedule, w.max_iters, early_stop=True, nms_num=w.nms_num,
                             nms_shift=w.nms_shift, oms_offset=w.oms_offset, msg_max=w.msg_max)
        info = w.info_bits_per_cw
        pools[cfg] = (pools[cfg], info)
    for mix, njobs in (("binary", 16), ("binary", 64), ("binary", 256), ("with_gf64", 16), ("with_gf64", 64),
                       ("with_gf64", 256)):
        jobs, bits = [], 0
        for _ in range(njobs):
            cfg = int(rng.choice([0, 1, 3], p=[0.5, 0.3, 0.2] if mix == "with_gf64" else [0.6, 0.4, 0.0]))
            size = int(np.exp(rng.uniform(0, np.log(257))))
            off = int(rng.integers(0, 512 - size + 1))
            x, info = pools[cfg]
            jobs.append((codes[cfg], prms[cfg], x[off:off + size]))
            bits += info * size
        stream = torch.cuda.current_stream()
        sp = int(stream.cuda_stream)
        # Both sides timed without Python marshalling: the ragged call reuses one prepared
        # job array, and the per-job loop makes one prepared C-ABI call per job; the
        # Python-level calls (outputs allocated and arguments marshalled every time) are
        # timed too.
        batch_pre = L.RaggedBatch(jobs)
        lib = L.lib()
        calls = []
        for h, prm, x in jobs:
            hh, ok, it = L._outputs(h, int(x.shape[0]), dev)
            calls.append((h.handle, ctypes.byref(prm), int(x.shape[0]), x.data_ptr(), hh.data_ptr(), ok.data_ptr(),
                          it.data_ptr(), None, sp, (hh, ok, it)))

        def run_ragged():
            batch_pre.run(stream)

        def run_loop():
            for c in calls:
                L._check(lib.ldpcx_decode(*c[:9]))

        def run_ragged_py():
            L.decode_ragged(jobs, stream=stream)

        def run_loop_py():
            for h, prm, x in jobs:
                L.decode(h, prm, x, stream=stream)

        res = {}
        for name, fn in (("ragged_one_launch", run_ragged), ("one_decode_per_job", run_loop),
                         ("ragged_python", run_ragged_py), ("per_job_python", run_loop_py)):
            for _ in range(2):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reps = 5
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            res[name] = (time.perf_counter() - t0) * 1e3 / reps
        print(json.dumps({"metric": "ragged batch vs one decode per job", "mix": mix, "jobs": njobs,
                          "codewords": sum(int(x.shape[0]) for _, _, x in jobs),
                          "ms_ragged": round(res["ragged_one_launch"], 3),
                          "ms_per_job_calls": round(res["one_decode_per_job"], 3),
                          "speedup": round(res["one_decode_per_job"] / res["ragged_one_launch"], 2),
                          "ms_ragged_python": round(res["ragged_python"], 3),
                          "ms_per_job_python": round(res["per_job_python"], 3),
                          "info_gbit_s_ragged": round(bits / (res["ragged_one_launch"] * 1e-3) / 1e9, 4)}),
              flush=True)


# ------------------------------------------------------------------ serving mix
SERVE_MIX = (0.4, 0.3, 0.1, 0.2)      # share of requests per code (n192, n2304, n64800, GF(64) n192)
SERVE_EBN0_CFG1 = (1.0, 1.5, 2.0, 2.5, 3.0)
SERVE_MAX_CW = 4096


def serve_pools(S, sizes):
    """Seeded input pools per (code, Eb/N0); a request takes a slice starting at a random
    offset (wrapping around), so its inputs are fixed by the serving seed alone."""
    pools = {}
    for cfg, size in sizes.items():
        ebs = SERVE_EBN0_CFG1 if cfg == 1 else (None,)
        for eb in ebs:
            w = S.workload(cfg, batch=size, ebn0_db=eb)
            _, llr = S.make_inputs(w, seed_offset=4200)
            pools[(cfg, eb)] = (w, np.ascontiguousarray(llr))
            print(f"serve: pool {w.name} Eb/N0 {w.ebn0_db} dB, {size} codewords", file=sys.stderr, flush=True)
    return pools


def serve_requests(pools, n, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(n):
        cfg = int(rng.choice(4, p=SERVE_MIX))
        size = int(np.floor(np.exp(rng.uniform(0.0, np.log(SERVE_MAX_CW + 1)))))
        size = max(1, min(SERVE_MAX_CW, size))
        eb = float(rng.choice(SERVE_EBN0_CFG1)) if cfg == 1 else None
        w, pool = pools[(cfg, eb)]
        off = int(rng.integers(0, pool.shape[0]))
        idx = (off + np.arange(size)) % pool.shape[0]
        reqs.append((cfg, w, np.ascontiguousarray(pool[idx])))
    return reqs


def serve_run(L, codes, prms, reqs, mode, budget, arrivals):
    """Submit reqs at the given arrival offsets (seconds; None = all at once) and wait for
    every one.  Returns per-request (latency_s, info_bits) and the makespan."""
    import threading
    srv = L.Server(hbm_budget=budget, max_inflight=4 if mode == "continuous" else 1, mode=mode)
    tickets = [None] * len(reqs)
    t_arr = [0.0] * len(reqs)
    start = time.perf_counter()

    def client():
        for i, (cfg, w, llr) in enumerate(reqs):
            if arrivals is not None:
                while True:
                    dt = start + arrivals[i] - time.perf_counter()
                    if dt <= 0:
                        break
                    time.sleep(min(dt, 0.002) if dt > 0.0005 else 0)
            t_arr[i] = time.perf_counter()
            tickets[i] = srv.submit(codes[cfg], prms[cfg], llr)

    th = threading.Thread(target=client)
    th.start()
    lat, bits = [], []
    for i, (cfg, w, llr) in enumerate(reqs):
        while tickets[i] is None:
            time.sleep(0.0002)
        _, _, _, (ts, ta, td) = srv.wait(tickets[i])
        # server clock: submit -> outputs in host memory; the client's own lag before
        # submit (arrival -> submit) is added from the client's clock
        lag = max(0.0, t_arr[i] - (start + (arrivals[i] if arrivals is not None else 0.0)))
        lat.append((td - ts) * 1e-6 + lag)
        bits.append(w.info_bits_per_cw * llr.shape[0])
    th.join()
    makespan = time.perf_counter() - start
    stats = srv.stats()
    srv.close()
    return np.array(lat), np.array(bits, dtype=np.float64), makespan, stats


def serve_main(args) -> None:
    import torch
    from paper_2508_03567_amd import ldpcx as L
    from paper_2508_03567_amd import synth as S

    torch.cuda.init()
    pools = serve_pools(S, {0: SERVE_MAX_CW, 1: SERVE_MAX_CW, 2: 1024, 3: SERVE_MAX_CW})
    codes, prms = {}, {}
    for cfg in range(4):
        w = S.workload(cfg)
        codes[cfg] = L.Code(w.code)
        prms[cfg] = L.params(w.rule, w.schedule, w.max_iters, early_stop=True, nms_num=w.nms_num,
                             nms_shift=w.nms_shift, oms_offset=w.oms_offset, msg_max=w.msg_max)
    budget = int(args.budget_gib * (1 << 30))
    modes = args.modes.split(",")
    n_meas, n_warm = args.requests, args.warm_requests
    # capacity of the continuous server on this mix: everything submitted at once
    cap_reqs = serve_requests(pools, max(200, n_meas // 4), seed=41)
    serve_run(L, codes, prms, cap_reqs[:20], "continuous", budget, None)  # warm-up
    _, bits, span, _ = serve_run(L, codes, prms, cap_reqs, "continuous", budget, None)
    capacity = len(cap_reqs) / span
    print(f"serve: capacity {capacity:.1f} requests/s ({bits.sum() / span / 1e9:.3f} Gbit/s info) on "
          f"{len(cap_reqs)} requests", file=sys.stderr, flush=True)
    reqs = serve_requests(pools, n_warm + n_meas, seed=42)
    for rho in [float(x) for x in args.rho.split(",")]:
        lam = rho * capacity
        rng = np.random.default_rng(int(rho * 1000) + 7)
        arrivals = np.cumsum(rng.exponential(1.0 / lam, size=len(reqs)))
        for mode in modes:
            lat, bits, span, st = serve_run(L, codes, prms, reqs, mode, budget, arrivals)
            m = lat[n_warm:]
            t_first = arrivals[n_warm]
            res = {"metric": "serving mix: p50/p99 latency and decoded info Gbit/s", "mode": mode, "rho": rho,
                   "arrival_rate_per_s": round(lam, 2), "requests": n_meas,
                   "p50_ms": round(float(np.percentile(m, 50)) * 1e3, 3),
                   "p99_ms": round(float(np.percentile(m, 99)) * 1e3, 3),
                   "mean_ms": round(float(m.mean()) * 1e3, 3),
                   "info_gbit_s": round(float(bits[n_warm:].sum()) / max(span - t_first, 1e-9) / 1e9, 4),
                   "launches": st["launches"], "peak_bytes": st["peak_bytes"], "budget_bytes": budget,
                   "capacity_req_s": round(capacity, 2), "data": "synthetic seeded BPSK/AWGN mix",
                   "mix": "40/30/10/20 % of n192 NMS / n2304 OMS layered (Eb/N0 1-3 dB) / n64800 NMS / GF(64) "
                          "n192 Min-Max, 1-4096 codewords log-uniform, early stop"}
            print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
