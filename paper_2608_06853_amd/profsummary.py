"""Readers of the rocprofv3 summaries kept in ``profiles/`` (HBM traffic per
dispatch, VALU counter rates), and the fingerprint of the sources each kernel
family is compiled from, so a reader can tell whether a committed summary still
describes the current kernel.
"""
from __future__ import annotations

import hashlib
import os

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
COMMON = ["af_device.h", "af_internal.h"]

# kernel family -> (symbol pattern, translation unit)
FAMILIES = {
    "table": (r"k_table[<(]", "k_table.hip"),
    "das_fwd": (r"k_das_fwd<", "k_das.hip"),
    "das_adj": (r"k_das_adj<", "k_das.hip"),
    "zero_tx": (r"k_zero_tx\(", "k_das.hip"),
    "das_rx": (r"k_das_rx<", "k_das.hip"),
    "loc": (r"k_loc\(", "k_das.hip"),
    "cmpe": (r"k_cmpe[<(]", "k_cmpe.hip"),
    "gscale": (r"k_gscale\(", "k_misc.hip"),
    "path_adj": (r"k_path_adj[<(]", "k_path.hip"),
    "path_chunk": (r"k_path_chunk\(", "k_path.hip"),
    "path_reduce": (r"k_path_reduce\(", "k_path.hip"),
    "prepare_grid": (r"k_prepare_grid\(", "k_misc.hip"),
    "finalize": (r"k_finalize\(", "k_misc.hip"),
    "grad_fold": (r"k_grad_fold\(", "k_misc.hip"),
    "sim_synth": (r"k_sim_synth\(", "k_sim.hip"),
    "sim_times": (r"k_sim_times\(", "k_sim.hip"),
    "conv_fwd": (r"k_conv_fwd\(", "k_cnn.hip"),
    "conv_bwd_data": (r"k_conv_bwd_data(_s2)?\(", "k_cnn.hip"),
    "conv_bwd_weight": (r"k_conv_bwd_weight\(", "k_cnn.hip"),
    "conv_wreduce": (r"k_conv_wreduce\(", "k_cnn.hip"),
    "conv_wsum": (r"k_conv_wsum\(", "k_cnn.hip"),
    "copy": (r"__amd_rocclr_copyBuffer", None),
}


def source_hash(family: str) -> str:
    tu = FAMILIES[family][1]
    if tu is None:
        return "-"
    h = hashlib.sha256()
    for f in [tu] + COMMON:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_counters(path: str) -> dict:
    """{family: (source hash, VALU instructions per CU per ns, lane utilisation,
    SQ_INSTS_VALU per dispatch)} from a counter summary (columns named by its last
    header line)."""
    out = {}
    cols = []
    with open(path) as f:
        for line in f:
            if line.startswith("# family"):
                cols = line[1:].split()
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            n_valu = float(p[cols.index("SQ_INSTS_VALU")]) if "SQ_INSTS_VALU" in cols else float("nan")
            out[p[0]] = (p[1], float(p[3]), float(p[4]), n_valu)
    return out


def read_traffic(path: str) -> dict:
    """{family: (source hash, bytes per dispatch)} from a traffic summary."""
    out = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            if len(p) == 6:
                out[p[0]] = (p[1], float(p[5]))
    return out
