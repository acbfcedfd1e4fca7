"""Full genotype-phenotype map of one lattice, streamed in sequence blocks.

    python -m paper_2008_05612_amd.fullmap --lattice 6x6 [--form blocked|gemm|popcount]
        [--symmetric] [--block-bits 30] [--neighbors] [--phi] [--table E_PP,E_PH,E_HP,E_HH]
        [--checkpoint FILE] [--json OUT]

Every step of 2^block_bits sequences is one library call; a progress line is
printed per step.  The default form is the block-factorised int8 form where
it applies (N >= 8; two-letter tables up to a 256-deep first product),
else the dense int8 form.  With --symmetric
only reversal-canonical work is scored (about half): canonical sequences
s <= reverse(s) for the dense and popcount forms (hp_enumerate_symmetric),
canonical blocks for the blocked form (hp_enumerate_symmetric_blocked); each
result is written at both s and reverse(s), and the steps run over canonical
indices.  The uint16 map stays resident on the device (2^36 x 2 B = 137 GB
for 6x6) unless --no-map is given.  With --symmetric and the blocked form the
canonical blocks are wide (1024 sequences, hp_enumerate_symmetric_wide)
where they apply.  With --checkpoint, the accumulated
designability is written after every step and a rerun resumes after the last
finished step (the map of skipped steps is then not available, so
--neighbors is refused on a resumed run).  --phi builds the whole phi_pq
matrix of Eq. 2 (dense counts on the device, n_class (n_class + 1) 8 bytes,
then compressed rows) and reports its size, its symmetry check and the
connected components of the phenotype graph (designable phenotypes joined
when a single mutation links them).

All device work goes through the C ABI (hp_enumerate, hp_enumerate_symmetric,
hp_enumerate_symmetric_blocked, hp_enumerate_symmetric_wide, hp_neighbors,
hp_phi_counts, hp_phi_sparse).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

from . import _binding as hp


def _parse_lattice(text: str):
    dims = [int(x) for x in text.lower().split("x")]
    while len(dims) < 3:
        dims.append(1)
    return tuple(dims)


def _load_checkpoint(path, dims, form, block_bits, n_class, symmetric, table, geometry):
    if not path or not os.path.exists(path):
        return None
    with open(path) as f:
        ck = json.load(f)
    if (tuple(ck["dims"]) != dims or ck["form"] != form or ck["block_bits"] != block_bits
            or len(ck["designability"]) != n_class or ck.get("symmetric", False) != symmetric
            or ck.get("table") != (list(table) if table else None)
            or ck.get("geometry", geometry) != geometry):
        raise ValueError("checkpoint %s is for another run" % path)
    return ck


def _save_checkpoint(path, dims, form, block_bits, symmetric, table, geometry, next_block, desig,
                     nondesign):
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump({"dims": list(dims), "form": form, "block_bits": block_bits,
                   "symmetric": symmetric, "table": list(table) if table else None,
                   "geometry": geometry,
                   "next_block": next_block,
                   "designability": [int(x) for x in desig], "nondesign": int(nondesign)}, f)
    os.replace(tmp, path)


def run(dims, form=None, block_bits=30, keep_map=True, neighbors=False,
        checkpoint=None, progress=print, device="cuda", symmetric=False, table=None,
        phi=False, fill=None):
    """Enumerate all 2^N sequences of the box; returns a summary dict (and the
    device map under key "map" when keep_map).  With `fill` (an int16 value
    that is no phenotype) the map starts filled with it and the summary
    counts the entries still holding it at the end ("unwritten")."""
    import numpy as np
    import torch

    s = hp.Structures(*dims, table=table)
    ws = s.workspace(device)
    N = s.N
    total = 1 << N
    if form is None:
        form = hp.FORM_BLOCKED_I8 if hp.hp_canonical_block_count(s) else hp.FORM_GEMM_I8
    # the blocked form's canonical blocks: wide (1024 sequences, the first
    # product shared by a workgroup) where they apply and the launch shape
    # allows, else blocks of 256
    wide_sym = (symmetric and form == hp.FORM_BLOCKED_I8 and hp.hp_wide_block_count(s) > 0
                and hp.hp_blocked_selected() in ((4, -1), (4, 3)))
    blocked_sym = symmetric and form == hp.FORM_BLOCKED_I8 and not wide_sym
    # indices to process: sequences, canonical sequences, or canonical blocks
    # of 256 or 1024 sequences; one step covers 2^block_bits sequences' worth
    if wide_sym:
        space = hp.hp_wide_block_count(s)
        block = 1 << max(0, min(block_bits, N) - 10)
        per_index = 1024
    elif blocked_sym:
        space = hp.hp_canonical_block_count(s)
        block = 1 << max(0, min(block_bits, N) - 8)
        per_index = 256
    else:
        space = hp.hp_canonical_count(s) if symmetric else total
        block = 1 << min(block_bits, N)
        per_index = 1
    geometry = "wide" if wide_sym else ("blocks256" if blocked_sym else "sequences")
    n_blocks = (space + block - 1) // block
    desig = torch.zeros(s.n_class, dtype=torch.int64, device=device)
    nond = torch.zeros(1, dtype=torch.int64, device=device)
    start_block = 0
    ck = _load_checkpoint(checkpoint, dims, form, block_bits, s.n_class, symmetric, table,
                          geometry)
    if ck:
        start_block = ck["next_block"]
        desig.copy_(torch.tensor(np.array(ck["designability"], dtype=np.uint64).view(np.int64)))
        nond.fill_(ck["nondesign"])
        if (neighbors or phi) and start_block > 0:
            raise ValueError("neighbour counts need the whole map; resume without "
                             "--neighbors / --phi")
        progress("resuming at block %d of %d" % (start_block, n_blocks))
    out = torch.empty(total, dtype=torch.int16, device=device) if keep_map else None
    if out is not None and fill is not None:
        out.fill_(fill)
    t0 = time.time()
    for b in range(start_block, n_blocks):
        lo, hi = b * block, min((b + 1) * block, space)
        tb = time.time()
        if wide_sym:
            hp.hp_enumerate_symmetric_wide(s, ws, lo, hi, out, None, desig, nond)
        elif blocked_sym:
            hp.hp_enumerate_symmetric_blocked(s, ws, lo, hi, out, None, desig, nond)
        elif symmetric:
            hp.hp_enumerate_symmetric(s, ws, form, lo, hi, out, None, desig, nond)
        else:
            hp.hp_enumerate(s, ws, form, lo, hi, out[lo:hi] if out is not None else None, None,
                            desig, nond)
        torch.cuda.synchronize()
        if checkpoint:
            _save_checkpoint(checkpoint, dims, form, block_bits, symmetric, table, geometry, b + 1,
                             desig.cpu().numpy().view(np.uint64), int(nond.item()))
        progress("block %d/%d [%d, %d) %.2f s" % (b + 1, n_blocks, lo, hi, time.time() - tb))
    wall = time.time() - t0
    d = desig.cpu().numpy().view(np.uint64)
    nd = int(nond.item())
    summary = {
        "lattice": "x".join(str(x) for x in dims if x > 1) or "1",
        "N": N, "sequences": total, "n_conf": s.n_conf, "n_class": s.n_class,
        "form": {hp.FORM_GEMM_I8: "gemm_i8", hp.FORM_BLOCKED_I8: "blocked_i8"}.get(form, "popcount"),
        "symmetric": symmetric, "geometry": geometry, "scored_sequences": space * per_index,
        "blocks": n_blocks, "block_sequences": block * per_index, "resumed_at_block": start_block,
        "wall_s": wall,
        "evals_per_s": (space - start_block * block) * per_index * s.n_conf / wall,
        "map_evals_per_s": ((space - start_block * block) * per_index * s.n_conf / wall *
                            (total / (space * per_index))),
        "designing": int(d.sum()), "nondesign": nd,
        "designable_classes": int((d > 0).sum()),
        "top_class": int(d.argmax()), "top_designability": int(d.max()),
        "designability_sha256": hashlib.sha256(d.astype("<u8").tobytes()).hexdigest(),
        "sum_check": int(d.sum()) + nd == total,
    }
    if out is not None and fill is not None:
        # counted in slices: a comparison over the whole 2^36-entry map at
        # once would need tens of GB of temporaries
        step = 1 << 28
        summary["unwritten"] = sum(int(torch.count_nonzero(out[lo:lo + step] == fill).item())
                                   for lo in range(0, total, step))
    if neighbors and out is not None:
        z = lambda n: torch.zeros(n, dtype=torch.int64, device=device)  # noqa: E731
        neu, dele, oth, row = z(s.n_class), z(s.n_class), z(s.n_class), z(s.n_class + 1)
        tn = time.time()
        hp.hp_neighbors(s, out, neu, dele, oth, summary["top_class"], row)
        torch.cuda.synchronize()
        summary["neighbors_s"] = time.time() - tn
        neu_h = neu.cpu().numpy().view(np.uint64)
        dele_h = dele.cpu().numpy().view(np.uint64)
        oth_h = oth.cpu().numpy().view(np.uint64)
        des = d > 0
        summary["neighbor_sum_check"] = bool(np.array_equal(neu_h + dele_h + oth_h,
                                                            np.uint64(N) * d))
        rho = neu_h[des] / (N * d[des]).astype(np.float64)
        null = d[des] / float(total)
        summary["robust_above_null_fraction"] = float((rho > null).mean())
        summary["mean_phi_del"] = float((dele_h[des] / (N * d[des]).astype(np.float64)).mean())
        summary["isolated_phenotypes"] = int((oth_h[des] == 0).sum())
        summary["phenotypes_connected_to_top"] = int((row[:s.n_class].cpu().numpy() > 0).sum())
        summary["_counts"] = (neu_h, dele_h, oth_h)
    if phi and out is not None:
        summary.update(_phi_summary(s, out, d, device))
    summary["_designability"] = d
    if out is not None:
        summary["map"] = out
    summary["_structs"] = s
    return summary


def _phi_summary(s, out, d, device):
    """The whole phi_pq matrix of the map: dense counts, compressed rows, the
    mutation-involution symmetry check and the phenotype graph's components."""
    import numpy as np
    import torch
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    n = s.n_class
    counts = torch.zeros((n, n + 1), dtype=torch.int64, device=device)
    torch.cuda.synchronize()
    t0 = time.time()
    hp.hp_phi_counts(s, out, counts)
    torch.cuda.synchronize()
    t_counts = time.time() - t0
    sq = counts[:, :n]
    symmetric = bool((sq == sq.t()).all().item())
    rp = torch.empty(n + 1, dtype=torch.int64, device=device)
    t0 = time.time()
    nnz = hp.hp_phi_sparse(s, counts, rp)
    cols = torch.empty(max(nnz, 1), dtype=torch.int32, device=device)
    vals = torch.empty(max(nnz, 1), dtype=torch.int64, device=device)
    hp.hp_phi_sparse(s, counts, rp, cols, vals)
    torch.cuda.synchronize()
    t_sparse = time.time() - t0
    del counts, sq
    rp_h = rp.cpu().numpy()
    p = cols[:nnz].cpu().numpy().astype(np.int64)
    q = np.repeat(np.arange(n), np.diff(rp_h))
    off = (p != q) & (p != n)
    des = d > 0
    g = coo_matrix((np.ones(int(off.sum()), np.int8), (q[off], p[off])), shape=(n, n)).tocsr()
    ncomp, lab = connected_components(g, directed=False)
    sizes = np.bincount(lab[des], minlength=ncomp)
    sizes = sizes[sizes > 0]
    return {
        "phi_counts_s": t_counts, "phi_sparse_s": t_sparse, "phi_nnz": int(nnz),
        "phi_dense_bytes": n * (n + 1) * 8, "phi_symmetric": symmetric,
        "phi_offdiag_links": int(off.sum()),
        "phenotype_graph_components": int(len(sizes)),
        "phenotype_graph_largest_component": int(sizes.max()) if len(sizes) else 0,
        "phenotype_graph_isolated": int((sizes == 1).sum()),
    }


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--lattice", default="6x6")
    ap.add_argument("--form", choices=["blocked", "gemm", "popcount"], default=None)
    ap.add_argument("--block-bits", type=int, default=30)
    ap.add_argument("--symmetric", action="store_true")
    ap.add_argument("--neighbors", action="store_true")
    ap.add_argument("--phi", action="store_true")
    ap.add_argument("--table", default=None,
                    help="two-letter contact energies E_PP,E_PH,E_HP,E_HH (integers; the "
                         "paper's Table 1 scaled by 10 is 0,-10,-10,-23); default pure HP")
    ap.add_argument("--no-map", action="store_true")
    ap.add_argument("--checkpoint")
    ap.add_argument("--json")
    a = ap.parse_args(argv)
    form = {None: None, "blocked": hp.FORM_BLOCKED_I8, "gemm": hp.FORM_GEMM_I8,
            "popcount": hp.FORM_POPCOUNT}[a.form]
    res = run(_parse_lattice(a.lattice), form, a.block_bits, keep_map=not a.no_map,
              neighbors=a.neighbors, phi=a.phi, checkpoint=a.checkpoint,
              progress=lambda m: print(m, flush=True), symmetric=a.symmetric,
              table=tuple(int(x) for x in a.table.split(",")) if a.table else None)
    pub = {k: v for k, v in res.items() if not k.startswith("_") and k != "map"}
    line = json.dumps(pub)
    print(line, flush=True)
    if a.json:
        with open(a.json, "w") as f:
            f.write(line + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
