"""Detection accuracy of the sketch against exact out-degrees (Sec. 5).

The paper scores a detector on a traffic with N true super points (hosts
whose number of distinct opposite hosts is at least theta) by

  FPR = N+ / N   (N+: reported hosts that are not super points)
  FNR = N- / N   (N-: super points that are not reported)
  TFR = FPR + FNR

and studies TFR while g runs from 256 to 4096 for several (r, k, alpha).
This module does the same on the synthetic windows: the sketch and its
restore run in the HIP library; the exact out-degree of every source comes
from a sort and two unique passes over the window's (src, dst) keys on the
device.

    python -m paper_1803_11449_amd.accuracy [--workload single_window_1m]
"""
from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np
import torch

from . import ddhf, traffic


def exact_out_degree(pairs: torch.Tensor):
    """(src, degree) of every source of a window: the number of distinct
    destinations it sent to. pairs: int32 [n, 2] on the device. Returns two
    int64 tensors on the device, src ascending."""
    if pairs.numel() == 0:
        e = torch.zeros(0, dtype=torch.int64, device=pairs.device)
        return e, e
    p = pairs.reshape(-1, 2).to(torch.int64) & 0xFFFFFFFF
    # the source's top bit is flipped so that signed order is unsigned order
    keys = torch.unique(((p[:, 0] ^ 0x80000000) << 32) | p[:, 1])   # distinct, sorted
    hi, deg = torch.unique_consecutive(keys >> 32, return_counts=True)
    return (hi & 0xFFFFFFFF) ^ 0x80000000, deg


def true_super_points(src: torch.Tensor, deg: torch.Tensor, theta: float) -> np.ndarray:
    """Hosts with at least theta distinct destinations (uint32, ascending)."""
    return src[deg.to(torch.float64) >= theta].cpu().numpy().astype(np.uint32)


def rates(reported, truth) -> dict:
    """FPR, FNR and TFR of a reported host list against the true super
    points (both sequences of addresses, any order, no duplicates)."""
    rep = np.unique(np.asarray(reported, dtype=np.uint32))
    tru = np.unique(np.asarray(truth, dtype=np.uint32))
    n = len(tru)
    n_plus = int(len(np.setdiff1d(rep, tru, assume_unique=True)))
    n_minus = int(len(np.setdiff1d(tru, rep, assume_unique=True)))
    fpr = n_plus / n if n else (0.0 if n_plus == 0 else math.inf)
    fnr = n_minus / n if n else 0.0
    return {"N": n, "reported": int(len(rep)), "N_plus": n_plus, "N_minus": n_minus,
            "FPR": fpr, "FNR": fnr, "TFR": fpr + fnr}


# parameter families of the g sweep: (r, k, alpha), each with (r-2)*alpha + k >= 32
FAMILIES = {"r5_k14": (5, 14, 6), "r4_k14": (4, 14, 9), "r6_k14": (6, 14, 5),
            "r5_k18": (5, 18, 5)}
G_SWEEP = (256, 512, 1024, 2048, 4096)


def detect(pairs: torch.Tensor, g: int, r: int, k: int, alpha: int, theta: float,
           seed: int = traffic.HASH_SEED, device: int = 0):
    """Reported hosts and the restore info of one window."""
    with ddhf.Sketch(g, k, r, alpha, seed, device=device) as sk:
        sk.update(pairs)
        try:
            recs, info = sk.restore(theta)
        except ddhf.SketchError as e:
            if e.code == ddhf.SKETCH_E_SATURATED:
                return None, {"saturated": True}
            raise
    return recs["ip"], info


def sweep(pairs: torch.Tensor, theta: float, families=None, gs=G_SWEEP, device: int = 0,
          truth=None) -> list:
    """One row per (family, g): the rates and the sketch's size."""
    if truth is None:
        truth = true_super_points(*exact_out_degree(pairs), theta)
    rows = []
    for name in families or FAMILIES:
        r, k, alpha = FAMILIES[name]
        for g in gs:
            ips, info = detect(pairs, g, r, k, alpha, theta, device=device)
            row = {"family": name, "g": g, "r": r, "k": k, "alpha": alpha,
                   "sketch_mib": (r << k) * g / 8 / 2**20}
            if ips is None:
                row.update({"saturated": True, "N": len(truth)})
            else:
                row.update(rates(ips, truth))
                row["psi"] = info["psi"]
            rows.append(row)
    return rows


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workload", default="single_window_1m",
                    choices=("single_window_1m", "large_window_100m", "stream_window"))
    ap.add_argument("--windows", type=int, default=3,
                    help="windows (seeds) per workload; the rates are summed over them")
    ap.add_argument("--theta", type=float, default=1024.0)
    ap.add_argument("--families", default=None,
                    help="comma-separated subset of " + ",".join(FAMILIES))
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        print("accuracy study needs a GPU", file=sys.stderr)
        return 2
    fams = args.families.split(",") if args.families else (
        ["r5_k14", "r4_k14", "r6_k14"] if args.workload == "single_window_1m" else ["r5_k18"])
    totals: dict = {}
    for w in range(args.windows):
        if args.workload == "single_window_1m":
            spec, seed = traffic.spec_single_window_1m(), traffic.config_seed(1, w)
        elif args.workload == "large_window_100m":
            spec, seed = traffic.spec_large_window_100m(), traffic.config_seed(2, w)
        else:
            spec, seed = traffic.spec_stream_window(w), traffic.config_seed(3, w)
        pairs = traffic.generate(spec, seed, device=torch.device("cuda:0")).pairs
        rows = sweep(pairs, args.theta, fams)
        for row in rows:
            key = (row["family"], row["g"])
            t = totals.setdefault(key, {**{k: row[k] for k in ("family", "g", "r", "k", "alpha",
                                                               "sketch_mib")},
                                        "N": 0, "N_plus": 0, "N_minus": 0, "saturated": 0})
            t["N"] += row["N"]
            if row.get("saturated"):
                t["saturated"] += 1
            else:
                t["N_plus"] += row["N_plus"]
                t["N_minus"] += row["N_minus"]
        del pairs
        torch.cuda.empty_cache()
        print(f"window {w} done", file=sys.stderr, flush=True)
    for t in totals.values():
        n = t["N"]
        t["FPR"] = t["N_plus"] / n if n else 0.0
        t["FNR"] = t["N_minus"] / n if n else 0.0
        t["TFR"] = t["FPR"] + t["FNR"]
        t.update({"workload": args.workload, "windows": args.windows, "theta": args.theta})
        print(json.dumps(t), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
