"""Readers for the hand-worked fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _hex_list(text):
    return np.array([int(t, 16) for t in text.split()], dtype=np.uint32)


def sort_cases():
    """Yield (name, i32, in_keys, out_keys, idx) from hand_cases.txt."""
    cases = []
    cur = None
    with open(os.path.join(GOLDEN, "hand_cases.txt")) as f:
        for line in f:
            line = line.rstrip("\n")
            if not line or line.startswith("#"):
                continue
            if line.startswith("case "):
                _, name, kind = line.split()
                cur = {"name": name, "i32": kind == "i32"}
                cases.append(cur)
            elif line.startswith("in:"):
                cur["in"] = _hex_list(line[3:])
            elif line.startswith("out:"):
                cur["out"] = _hex_list(line[4:])
            elif line.startswith("idx:"):
                cur["idx"] = np.array([int(t) for t in line[4:].split()], dtype=np.uint32)
    return [(c["name"], c["i32"], c["in"], c["out"], c["idx"]) for c in cases]


def partition_cases():
    """Return (keys, run_offsets, [(r, c_vector), ...]) from hand_partitions.txt."""
    runs = None
    splits = []
    with open(os.path.join(GOLDEN, "hand_partitions.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("runs:"):
                runs = [[int(t) for t in part.split()] for part in line[5:].split("|")]
            elif line.startswith("r="):
                lhs, rhs = line.split(":")
                splits.append((int(lhs[2:]), [int(t) for t in rhs.split()]))
    keys = np.array([k for run in runs for k in run], dtype=np.uint32)
    offs = np.cumsum([0] + [len(r) for r in runs]).astype(np.uint64)
    return keys, offs, splits


def sort_cases_u64():
    """Yield (name, i64, in_keys, out_keys, idx) from hand_cases_u64.txt."""
    cases = []
    cur = None
    with open(os.path.join(GOLDEN, "hand_cases_u64.txt")) as f:
        for line in f:
            line = line.rstrip("\n")
            if not line or line.startswith("#"):
                continue
            if line.startswith("case "):
                _, name, kind = line.split()
                cur = {"name": name, "i64": kind == "i64"}
                cases.append(cur)
            elif line.startswith("in:"):
                cur["in"] = np.array([int(t, 16) for t in line[3:].split()], dtype=np.uint64)
            elif line.startswith("out:"):
                cur["out"] = np.array([int(t, 16) for t in line[4:].split()], dtype=np.uint64)
            elif line.startswith("idx:"):
                cur["idx"] = np.array([int(t) for t in line[4:].split()], dtype=np.uint64)
    return [(c["name"], c["i64"], c["in"], c["out"], c["idx"]) for c in cases]
