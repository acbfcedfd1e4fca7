#!/usr/bin/env python3
"""Benchmark of the HP genotype-phenotype map hot path on one MI355X.

One step = the whole path over the 3x3x3 cube: ground states of all 2^27
sequences against all 103346 conformations (block-factorised int8-MFMA form:
energy products, min/unique/argmin epilogue, designability atomics), then the
single-mutation neighbour counts (with the phi row of the most designable
phenotype) and the neutral-network union-find over the full map.  Structures
are enumerated and uploaded once before timing; all inputs are resident in
HBM.

Roofline of the dominant kernel: the method's work per (sequence,
conformation) pair is nbp contact products h_i h_j and their sum (Eq. 1; 28
contacts per 3x3x3 conformation), i.e. 2 nbp integer operations, priced
against the dense int8 MFMA peak of the contraction's data type.  What the
kernel issues instead (depth-32 products, the first product per block, the
vector-ALU test of each product) is reported under "extra".

Prints ONE JSON line.  Extra measurements (dense int8 and popcount forms, the
full 6x6 map, the mixed-lattice batch, the sampling mode, per-kernel times) go
in the same line under "extra".
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("seq×structure evals/s + full-map wall time (3×3×3, 6×6); "
          "% int8 MFMA peak")
PEAK_INT8_TOPS = 5000.0          # MI355X dense int8 MFMA, TOP/s
PEAK_VALU_TOPS = 256 * 2.4e9 * 64 / 1e12   # 32-bit VALU lane-ops/s: 256 CU x 64 lanes/clk x 2.4 GHz
# with two VALU instructions issued per quad-cycle (gfx950 dual issue; the
# popcount form's two-operand instructions reach it)
PEAK_VALU_DUAL_TOPS = 2 * PEAK_VALU_TOPS
# sources of the blocked kernel: a recorded counter summary only counts for
# the build it was taken on
KERNEL_SOURCES = ["gemm_blk.h", "gemm_blk_kb5.hip", "gemm_blk.hip", "gemm_body.h",
                  "device_common.h", "kernels.h", "hp_internal.h"]
# the designability histogram of the full pure-HP 6x6 map, as first computed
# (SHA-256 of the uint64 little-endian counts); later runs must reproduce it
SHA_6X6_PURE_HP = "250821539f228f1daeea4954d24c83dda5880d750ad6d9911f2eff764972e261"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2008_05612_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--autotune", action="store_true",
                    help="time every launch shape of the blocked form and every tile shape of "
                         "the dense form first, and use the fastest")
    ap.add_argument("--nw", type=int, default=4,
                    help="waves per workgroup of the blocked form (2, 4 or 8)")
    ap.add_argument("--blk-mode", type=int, default=-1,
                    help="staging mode of the blocked form (0 double-buffered, 1 pipelined, "
                         "2 second operand in LDS, 3 wide blocks, -1 wide blocks where they "
                         "apply, else by product depth)")
    ap.add_argument("--profile", action="store_true",
                    help="profiling run: no extras, no CPU baseline, plus one dense-form "
                         "full map and a 256 MiB device copy used to calibrate the HBM byte "
                         "counters")
    return ap.parse_args()


class Timer:
    """Event pair on torch's current stream, which is the stream every
    library call in this script is enqueued on."""

    def __init__(self):
        import torch
        self.a = torch.cuda.Event(enable_timing=True)
        self.b = torch.cuda.Event(enable_timing=True)

    def start(self):
        self.a.record()

    def stop(self):
        self.b.record()

    def ms(self):
        return self.a.elapsed_time(self.b)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the sequence range would shard across GPUs; see the design notes).",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2008_05612_amd as hp

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    dims = (3, 3, 3)
    t0 = time.time()
    s = hp.Structures(*dims)
    ws = s.workspace()
    t_struct = time.time() - t0
    N, total, n_conf = s.N, 1 << s.N, s.n_conf
    if args.profile:
        args.no_extra = True
        args.no_cpu_baseline = True
    tune_ms = None
    hp.hp_blocked_select(args.nw, args.blk_mode)
    nw = args.nw
    # the staging the library takes for mode -1: wide blocks where they apply
    # (pure pair energies, N >= 10, 4 or 8 waves), else by product depth
    wide = s.unary_rows == 0 and s.N >= 10 and nw in (4, 8)
    blk_mode = (args.blk_mode if args.blk_mode >= 0 and (args.blk_mode != 3 or wide)
                else (3 if wide else (2 if s.K_pad <= 192 else 0)))
    if args.autotune:
        _, tune_ms = hp.hp_autotune(s, ws, 0, 1 << 20, repeats=2)
        (nw, blk_mode), blk_ms = hp.hp_autotune_blocked(s, ws, 0, 1 << 22, repeats=2)
        tune_ms = {"dense": tune_ms, "blocked": blk_ms}
    # wide blocks with 8 waves (the default, or --nw 8): the whole map, one
    # range cut at a multiple of 2^17, takes blocks of 2048 sequences where
    # N >= 17; --nw 4 --blk-mode 3 keeps blocks of 1024 on 4 waves
    wide8 = blk_mode == 3 and (args.blk_mode < 0 or nw == 8) and s.N >= 17
    kname = ("k_gemm_wide_w8<%d>" % (s.K_pad // 32) if wide8
             else "k_gemm_wide<%d>" % (s.K_pad // 32) if blk_mode == 3
             else "k_gemm_blk<%d,%d,%d>" % (s.K_pad // 32, nw, blk_mode))
    pairs = total * n_conf

    out = torch.empty(total, dtype=torch.int16, device=dev)
    desig = torch.zeros(s.n_class, dtype=torch.int64, device=dev)
    nond = torch.zeros(1, dtype=torch.int64, device=dev)
    z = lambda n: torch.zeros(n, dtype=torch.int64, device=dev)  # noqa: E731
    neu, dele, oth, row = z(s.n_class), z(s.n_class), z(s.n_class), z(s.n_class + 1)
    labels = torch.empty(total, dtype=torch.int32, device=dev)
    csize = torch.empty(total, dtype=torch.int32, device=dev)
    ncomp = torch.empty(s.n_class, dtype=torch.int32, device=dev)
    largest = torch.empty(s.n_class, dtype=torch.int32, device=dev)

    timers = {"enumerate": Timer(), "neighbors": Timer(), "components": Timer()}
    kms = {k: [] for k in timers}
    top = -1

    def step(phi_q):
        for t in (desig, nond, neu, dele, oth, row):
            t.zero_()
        timers["enumerate"].start()
        hp.hp_enumerate(s, ws, hp.FORM_BLOCKED_I8, 0, total, out, None, desig, nond)
        timers["enumerate"].stop()
        timers["neighbors"].start()
        hp.hp_neighbors(s, out, neu, dele, oth, phi_q, row if phi_q >= 0 else None)
        timers["neighbors"].stop()
        timers["components"].start()
        hp.hp_components(s, out, labels, csize, ncomp, largest)
        timers["components"].stop()

    for i in range(max(args.warmup, 1)):
        step(top)
        torch.cuda.synchronize()
        if top < 0:
            top = int(torch.argmax(desig).item())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in range(args.steps):
        step(top)
        torch.cuda.synchronize()
        for k, t in timers.items():
            kms[k].append(t.ms())
    t2 = time.perf_counter()
    ms_step = (t2 - t1) * 1e3 / args.steps

    d = desig.cpu().numpy().view(np.uint64)
    nd = int(nond.item())
    assert int(d.sum()) + nd == total, "designability + deleterious != 2^N"

    enum_ms = float(np.mean(kms["enumerate"]))
    # the method's work: nbp contact products h_i h_j and their sum per pair
    method_ops = 2.0 * s.nbp * pairs
    achieved_tops = method_ops / (enum_ms * 1e-3) / 1e12
    # MFMA work the blocked form issues: one depth-32 product per pair, plus
    # the per-block first product (K_pad deep, 32 virtual rows) per
    # conformation tile, once per block of 256 sequences, or of 1024 or 2048
    # for wide blocks
    n_tiles = (n_conf + 31) // 32
    block_seqs = 2048 if wide8 else 1024 if blk_mode == 3 else 256
    blk_mfma_ops = (2.0 * 32 * pairs +
                    2.0 * s.K_pad * 32 * 32 * n_tiles * (total // block_seqs))
    evals_per_s = pairs / (ms_step * 1e-3)
    src_hash = kernel_source_hash()

    result = {
        "metric": METRIC,
        "value": evals_per_s,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "data": "synthetic",
        "config": {
            "workload": "3x3x3 full map: all 2^27 sequences x 103346 conformations "
                        "(block-factorised int8-MFMA form) + single-mutation neighbour "
                        "counts + union-find",
            "lattice": "3x3x3", "N": N, "sequences": total, "n_conf": n_conf,
            "n_class": s.n_class, "K": s.K, "K_pad": s.K_pad, "nbp": s.nbp,
            "form": "blocked_i8", "waves_per_workgroup": 8 if wide8 else nw,
            "staging_mode": blk_mode, "block_sequences": block_seqs,
        },
        "roofline": {
            "bound": "mfma",
            "achieved": achieved_tops,
            "peak": PEAK_INT8_TOPS,
            "unit": "TOP/s",
            "frac": achieved_tops / PEAK_INT8_TOPS,
            "traffic": recorded_traffic(kname, src_hash),
            "kernel": kname + " (hp_enumerate, blocked int8 form)",
            "ops_per_unit": 2 * s.nbp,
            "unit_of_work": "one (sequence, conformation) pair: nbp contact products and "
                            "their sum (Eq. 1)",
            "units_per_launch": pairs,
            "launch_ms": enum_ms,
        },
    }
    extra = {
        "full_map_ms_3x3x3": ms_step,
        "kernel_ms": {k: float(np.mean(v)) for k, v in kms.items()},
        "enumerate_evals_per_s": pairs / (enum_ms * 1e-3),
        # matrix-pipe utilisation: what the blocked kernel issues (depth-32
        # products for every pair plus the per-block first product)
        "blocked_mfma_pipe_frac": blk_mfma_ops / (enum_ms * 1e-3) / 1e12 / PEAK_INT8_TOPS,
        "blocked_mfma_ops_per_pair": blk_mfma_ops / pairs,
        "kernel_source_sha": src_hash,
        "designing_fraction": float(d.sum()) / total,
        "top_class": top,
        "top_designability": int(d[top]),
        "structures_s": t_struct,
        "autotune_ms_per_shape": tune_ms,
    }
    extra.update(recorded_issue(kname, src_hash))
    if not args.no_extra:
        extra.update(extra_measurements(hp, s, ws, dev, out))
    if args.profile:
        # the dense int8 form over the same full map, once, so that profiles of
        # this run cover both int8 kernels
        hp.hp_enumerate(s, ws, hp.FORM_GEMM_I8, 0, total, out)
        torch.cuda.synchronize()
        # a plain copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE counters
        a = torch.empty(1 << 28, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        a.fill_(1)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        extra["calibration_copy_bytes"] = a.numel()
    result["extra"] = extra
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(dims, args.cpu_seconds)
    print(json.dumps(result), flush=True)


HP1996_X10 = (0, -10, -10, -23)   # Table 1 energies scaled by 10: E_PP, E_PH, E_HP, E_HH


def _summary_fields(name):
    fields = {}
    try:
        for line in open(os.path.join(ROOT, "profiles", name)):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    except OSError:
        pass
    return fields


def _summary_name(kname, what):
    """profiles/ file of the counter summary `what` for kernel `kname`
    (k_gemm_wide<KB>, k_gemm_wide_w8<KB> or k_gemm_blk<KB,NW,MODE>) on the
    3x3x3 map."""
    family = "k_gemm_wide" if kname.startswith("k_gemm_wide") else "k_gemm_blk"
    return "%s_3x3x3_%s.txt" % (family, what)


def recorded_traffic(kname, src_hash):
    """HBM bytes per full-map launch of `kname`, from the calibrated
    FETCH_SIZE / WRITE_SIZE counter summary of the blocked kernel in
    profiles/, or None when that summary is for another kernel or another
    build of its sources."""
    f = _summary_fields(_summary_name(kname, "hbm_traffic"))
    if f.get("kernel") != kname or f.get("source_sha") != src_hash:
        return None
    try:
        return float(f["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def recorded_issue(kname, src_hash):
    """Vector-ALU and matrix-pipe issue figures of the blocked kernel from
    its counter summary in profiles/ (same build only)."""
    f = _summary_fields(_summary_name(kname, "issue_counters"))
    if f.get("kernel") != kname or f.get("source_sha") != src_hash:
        return {"blocked_issue_counters": None}
    keep = ("valu_per_wave_tile", "mfma_per_wave_tile", "valu_issue_per_simd_quad_cycle",
            "mfma_busy", "dual_issue")
    return {"blocked_issue_counters": {k: float(f[k]) for k in keep if k in f}}


def extra_measurements(hp, s, ws, dev, blocked_map):
    """The whole phi_pq matrix of the full 3x3x3 map (dense counts and
    compressed rows), the paper's own timed workload (Table 1 energies,
    sampled sequences) on 3x3x3 and 6x6, the dense int8 form over the same
    full 3x3x3 map (its fractions of the int8 MFMA peak, and a bit-exact
    comparison with the blocked form's map), the popcount form on a 2^24
    slice, the sampling mode on both lattices, one 2^28 block of the 6x6 map
    in all three forms, the full 6x6 map (measured), and the mixed-lattice
    batch."""
    import numpy as np
    import torch
    res = {}
    t = Timer()
    total = 1 << s.N
    # the whole phi_pq matrix of the map (Eq. 2): dense counts, then
    # compressed rows
    n = s.n_class
    counts = torch.zeros((n, n + 1), dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    t.start()
    hp.hp_phi_counts(s, blocked_map, counts)
    t.stop()
    torch.cuda.synchronize()
    res["phi_counts_ms_3x3x3"] = t.ms()
    rp = torch.empty(n + 1, dtype=torch.int64, device=dev)
    t0 = time.perf_counter()
    nnz = hp.hp_phi_sparse(s, counts, rp)
    cols = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
    vals = torch.empty(max(nnz, 1), dtype=torch.int64, device=dev)
    hp.hp_phi_sparse(s, counts, rp, cols, vals)
    torch.cuda.synchronize()
    res["phi_sparse_ms_3x3x3"] = (time.perf_counter() - t0) * 1e3
    res["phi_matrix_nnz_3x3x3"] = nnz
    res["phi_matrix_dense_bytes_3x3x3"] = counts.numel() * 8
    del counts, cols, vals, rp
    dense = torch.empty(total, dtype=torch.int16, device=dev)
    hp.hp_enumerate(s, ws, hp.FORM_GEMM_I8, 0, 1 << 16, dense)
    torch.cuda.synchronize()
    t.start()
    hp.hp_enumerate(s, ws, hp.FORM_GEMM_I8, 0, total, dense)
    t.stop()
    torch.cuda.synchronize()
    T, NW, mode = hp.hp_gemm_shapes(s.K_pad)[hp.hp_gemm_selected(s.K_pad)]
    res["dense_gemm_i8_shape"] = {"T": T, "NW": NW, "mode": mode}
    res["dense_gemm_i8_full_map_ms_3x3x3"] = t.ms()
    res["dense_gemm_i8_evals_per_s"] = total * s.n_conf / (t.ms() * 1e-3)
    # the method's work (2 nbp per pair) and the matrix pipe's (2 K_pad per
    # pair: a dense product over every odd-separation pair row)
    res["dense_gemm_i8_method_frac"] = (2.0 * s.nbp * total * s.n_conf / (t.ms() * 1e-3) /
                                        1e12 / PEAK_INT8_TOPS)
    res["dense_gemm_i8_mfma_pipe_frac"] = (2.0 * s.K_pad * total * s.n_conf /
                                           (t.ms() * 1e-3) / 1e12 / PEAK_INT8_TOPS)
    res["blocked_map_equals_dense_map"] = bool(torch.equal(dense, blocked_map))
    # the same full map from reversal-canonical blocks only (about half the work)
    nb = hp.hp_canonical_block_count(s)
    dsym = torch.zeros(s.n_class, dtype=torch.int64, device=dev)
    hp.hp_enumerate_symmetric_blocked(s, ws, 0, 1024, dense, None, dsym)
    torch.cuda.synchronize()
    dsym.zero_()
    t.start()
    hp.hp_enumerate_symmetric_blocked(s, ws, 0, nb, dense, None, dsym)
    t.stop()
    torch.cuda.synchronize()
    res["symmetric_blocked_full_map_ms_3x3x3"] = t.ms()
    res["symmetric_blocked_map_equals_blocked_map"] = bool(torch.equal(dense, blocked_map))
    # ... and from reversal-canonical wide blocks (1024 sequences each)
    nw_ = hp.hp_wide_block_count(s)
    if nw_:
        dsym.zero_()
        hp.hp_enumerate_symmetric_wide(s, ws, 0, 256, dense, None, dsym)
        torch.cuda.synchronize()
        dense.fill_(-2)
        dsym.zero_()
        t.start()
        hp.hp_enumerate_symmetric_wide(s, ws, 0, nw_, dense, None, dsym)
        t.stop()
        torch.cuda.synchronize()
        res["symmetric_wide_full_map_ms_3x3x3"] = t.ms()
        res["symmetric_wide_map_equals_blocked_map"] = bool(torch.equal(dense, blocked_map))
    del dense
    n = 1 << 24
    for form, name in ((hp.FORM_POPCOUNT, "popcount"), (hp.FORM_BLOCKED_I8, "blocked_i8")):
        hp.hp_enumerate(s, ws, form, 0, 1 << 16)
        torch.cuda.synchronize()
        t.start()
        hp.hp_enumerate(s, ws, form, 0, n)
        t.stop()
        torch.cuda.synchronize()
        res["3x3x3_slice_%s_evals_per_s" % name] = n * s.n_conf / (t.ms() * 1e-3)
    res["blocked_over_popcount_3x3x3"] = (res["3x3x3_slice_blocked_i8_evals_per_s"] /
                                          res["3x3x3_slice_popcount_evals_per_s"])
    res["dense_over_popcount_3x3x3"] = (res["dense_gemm_i8_evals_per_s"] /
                                        res["3x3x3_slice_popcount_evals_per_s"])
    # the popcount loop issues 2W + 4 VALU instructions per pair (W ANDs, W
    # bit counts, 4 for the key and top-2 update); its mix dual-issues
    res["popcount_valu_frac_3x3x3"] = (res["3x3x3_slice_popcount_evals_per_s"] *
                                       (2 * s.W + 4) / (PEAK_VALU_DUAL_TOPS * 1e12))
    # sampling mode (device-side draws): one launch of 2^14 draws -- the
    # launch size of the paper's sampling runs -- and one of 2^24; the
    # per-sequence time is the unit of the paper's CPU/GPU comparison table
    for nd_, name in ((1 << 14, "2^14"), (1 << 24, "2^24")):
        hp.hp_sample(s, ws, hp.FORM_GEMM_I8, 1, 0, 1 << 14, 1)
        torch.cuda.synchronize()
        t.start()
        hp.hp_sample(s, ws, hp.FORM_GEMM_I8, 0x2008056120, 0, nd_, 1)
        t.stop()
        torch.cuda.synchronize()
        sec = t.ms() * 1e-3
        res["3x3x3_sample_%s_evals_per_s" % name] = nd_ * s.n_conf / sec
        res["3x3x3_sample_%s_s_per_sequence" % name] = sec / nd_
    # the paper's timed workload itself: Table 1 energies (x10), random
    # sequences, 2^14 per launch, on both lattices of its CPU/GPU table
    for dims in ((3, 3, 3), (6, 6, 1)):
        sh = hp.Structures(*dims, table=HP1996_X10)
        wsh = sh.workspace()
        name = "x".join(str(x) for x in dims if x > 1)
        if hp.hp_canonical_block_count(sh):
            # the full map with these energies (the map the paper's printed
            # statistics come from), blocked form
            d96 = torch.zeros(sh.n_class, dtype=torch.int64, device=dev)
            hp.hp_enumerate(sh, wsh, hp.FORM_BLOCKED_I8, 0, 1 << 16)
            torch.cuda.synchronize()
            t.start()
            hp.hp_enumerate(sh, wsh, hp.FORM_BLOCKED_I8, 0, 1 << sh.N, None, None, d96)
            t.stop()
            torch.cuda.synchronize()
            res["%s_hp1996_full_map_ms_blocked" % name] = t.ms()
            res["%s_hp1996_designing_fraction" % name] = float(d96.sum().item()) / (1 << sh.N)
            del d96
        hp.hp_sample(sh, wsh, hp.FORM_GEMM_I8, 1, 0, 1 << 14, 1)
        torch.cuda.synchronize()
        for nd_, tag in ((1 << 14, "2^14"), (1 << 22, "2^22")):
            t.start()
            hp.hp_sample(sh, wsh, hp.FORM_GEMM_I8, 0x2008056120, 0, nd_, 1)
            t.stop()
            torch.cuda.synchronize()
            sec = t.ms() * 1e-3
            res["%s_hp1996_sample_%s_s_per_sequence" % (name, tag)] = sec / nd_
            res["%s_hp1996_sample_%s_evals_per_s" % (name, tag)] = nd_ * sh.n_conf / sec
        del wsh, sh
    s6 = hp.Structures(6, 6, 1)
    ws6 = s6.workspace()
    hp.hp_sample(s6, ws6, hp.FORM_GEMM_I8, 1, 0, 1 << 14, 1)
    torch.cuda.synchronize()
    t.start()
    hp.hp_sample(s6, ws6, hp.FORM_GEMM_I8, 0x2008056120, 0, 1 << 22, 1)
    t.stop()
    torch.cuda.synchronize()
    res["6x6_sample_2^22_evals_per_s"] = (1 << 22) * s6.n_conf / (t.ms() * 1e-3)
    res["6x6_sample_2^22_s_per_sequence"] = t.ms() * 1e-3 / (1 << 22)
    n6 = 1 << 28
    d6 = torch.zeros(s6.n_class, dtype=torch.int64, device=dev)
    nb6 = hp.hp_canonical_block_count(s6)
    for form, name, nn in ((hp.FORM_BLOCKED_I8, "blocked_i8", n6), (hp.FORM_GEMM_I8, "gemm_i8", n6),
                           (hp.FORM_POPCOUNT, "popcount", n6 // 4)):
        hp.hp_enumerate(s6, ws6, form, 0, 1 << 16, None, None, d6)
        torch.cuda.synchronize()
        t.start()
        hp.hp_enumerate(s6, ws6, form, 0, nn, None, None, d6)
        t.stop()
        torch.cuda.synchronize()
        rate = nn * s6.n_conf / (t.ms() * 1e-3)
        res["6x6_block_%s_evals_per_s" % name] = rate
    res["6x6_gemm_i8_mfma_pipe_frac"] = (res["6x6_block_gemm_i8_evals_per_s"] * 2 * s6.K_pad /
                                         (PEAK_INT8_TOPS * 1e12))
    res["6x6_blocked_method_frac"] = (res["6x6_block_blocked_i8_evals_per_s"] * 2 * s6.nbp /
                                      (PEAK_INT8_TOPS * 1e12))
    del d6
    # the full 6x6 map, measured: every canonical wide block of the blocked
    # form in one call (the library cuts it into launches of 2^30
    # sequences); the map itself is not kept (137 GB), its designability
    # histogram is hashed
    d6 = torch.zeros(s6.n_class, dtype=torch.int64, device=dev)
    nd6 = torch.zeros(1, dtype=torch.int64, device=dev)
    nw6 = hp.hp_wide_block_count(s6)
    print("bench: full 6x6 map (%d canonical wide blocks)" % nw6, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if nw6:
        hp.hp_enumerate_symmetric_wide(s6, ws6, 0, nw6, None, None, d6, nd6)
    else:
        hp.hp_enumerate_symmetric_blocked(s6, ws6, 0, nb6, None, None, d6, nd6)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    res["6x6_full_map_geometry"] = "canonical wide blocks" if nw6 else "canonical blocks of 256"
    h6 = d6.cpu().numpy().view(np.uint64)
    sha6 = hashlib.sha256(h6.astype("<u8").tobytes()).hexdigest()
    res["6x6_full_map_s"] = sec
    res["6x6_full_map_map_evals_per_s"] = (1 << 36) * s6.n_conf / sec
    res["6x6_full_map_designability_sha256"] = sha6
    res["6x6_full_map_sha_matches_first_run"] = sha6 == SHA_6X6_PURE_HP
    res["6x6_full_map_sum_check"] = int(h6.sum()) + int(nd6.item()) == 1 << 36
    res["6x6_full_map_designing"] = int(h6.sum())
    del d6, nd6, ws6, s6
    res.update(mixed_batch(hp, dev))
    return res


def mixed_batch(hp, dev):
    """The mixed-lattice batch at its full sizes (4x4, 5x5, 2x3x4 and 3x3x3,
    every sequence of each): one captured hipGraph replay against the same
    jobs as separate hp_enumerate calls, blocked form."""
    import torch
    jobs, outs, sizes = [], [], {}
    for dims in ((4, 4, 1), (5, 5, 1), (2, 3, 4), (3, 3, 3)):
        s = hp.Structures(*dims)
        ws = s.workspace()
        n = 1 << s.N
        o = torch.empty(n, dtype=torch.int16, device=dev)
        d = torch.zeros(s.n_class, dtype=torch.int64, device=dev)
        nd = torch.zeros(1, dtype=torch.int64, device=dev)
        jobs.append(hp.Job(s, ws, 0, n, o, None, d, nd))
        outs.append((s, ws, o, d, nd))
        sizes["x".join(str(x) for x in dims if x > 1)] = n * s.n_conf
    bws = torch.zeros(hp._binding.batch_workspace_bytes(len(jobs)), dtype=torch.uint8,
                      device=dev)
    g = hp.hp_graph_capture_batch(jobs, hp.FORM_BLOCKED_I8, bws)
    g.launch()
    torch.cuda.synchronize()
    t = Timer()
    t.start()
    g.launch()
    t.stop()
    torch.cuda.synchronize()
    graph_ms = t.ms()
    t.start()
    for s, ws, o, d, nd in outs:
        hp.hp_enumerate(s, ws, hp.FORM_BLOCKED_I8, 0, 1 << s.N, o, None, d, nd)
    t.stop()
    torch.cuda.synchronize()
    pairs = sum(sizes.values())
    return {"mixed_batch_graph_ms": graph_ms, "mixed_batch_separate_launches_ms": t.ms(),
            "mixed_batch_pairs": pairs, "mixed_batch_evals_per_s": pairs / (graph_ms * 1e-3),
            "mixed_batch_jobs": sizes}


def host_cpu():
    """CPU model, physical cores and hardware threads of this host."""
    model, cores = None, set()
    try:
        phys = core = None
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k == "model name" and model is None:
                model = v
            elif k == "physical id":
                phys = v
            elif k == "core id":
                core = v
            elif not k and phys is not None:
                cores.add((phys, core))
                phys = core = None
    except OSError:
        pass
    return {"model": model, "physical_cores": len(cores) or None,
            "hardware_threads": os.cpu_count(),
            "threads_available": len(os.sched_getaffinity(0))}


def _oracle_rate(oracle, st, lo, n):
    t0 = time.perf_counter()
    oracle.ground_states(st, lo, lo + n)
    dt = time.perf_counter() - t0
    return n * st.n_conf / dt, dt


def cpu_baseline(dims, seconds):
    """The oracle (plain C, OpenMP over sequences) on a bounded window of the
    same workload, on this host's cores (all threads and one thread), plus
    the other lattices of the same workload family: the full 4x4 map, a 5x5
    window and a 6x6 window; full-map times extrapolated from the rates."""
    import oracle
    st = oracle.structures(*dims)
    lo = 0
    n = 4096          # enough to keep every host thread busy while calibrating
    _, dt = _oracle_rate(oracle, st, lo, n)
    n = int(max(4096, min(1 << 22, n * seconds / max(dt, 1e-3))))
    rate, dt = _oracle_rate(oracle, st, lo, n)
    threads = oracle.num_threads()
    # one thread on a smaller sample of the same window
    oracle.set_num_threads(1)
    n1 = max(64, n // (4 * threads))
    rate1, dt1 = _oracle_rate(oracle, st, lo, n1)
    oracle.set_num_threads(threads)
    # the other lattices: 4x4 whole, 5x5 and 6x6 windows sized to a few seconds
    other = {}
    for d2, cap in (((4, 4, 1), 1 << 16), ((5, 5, 1), 1 << 22), ((6, 6, 1), 1 << 16)):
        st2 = oracle.structures(*d2)
        n2 = min(cap, 1 << 12)
        _, t2 = _oracle_rate(oracle, st2, 0, n2)
        n2 = int(max(n2, min(cap, n2 * 3.0 / max(t2, 1e-3))))
        r2, t2 = _oracle_rate(oracle, st2, 0, n2)
        name = "x".join(str(x) for x in d2 if x > 1)
        other[name] = {"evals_per_s": r2, "sample": "sequences [0, %d) x all %d conformations, "
                       "%.2f s" % (n2, st2.n_conf, t2),
                       "full_map_s_extrapolated": (1 << st2.N) * st2.n_conf / r2}
    return {"value": rate, "unit": "evals/s", "cores": threads,
            "kind": "oracle",
            "sample": "3x3x3, sequences [0, %d) x all %d conformations, %.1f s on %d threads"
                      % (n, st.n_conf, dt, threads),
            "host": host_cpu(),
            "value_1_thread": rate1,
            "sample_1_thread": "sequences [0, %d), %.1f s" % (n1, dt1),
            "full_map_s_extrapolated_3x3x3": (1 << st.N) * st.n_conf / rate,
            "other_lattices": other}


if __name__ == "__main__":
    main()
