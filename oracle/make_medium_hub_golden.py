"""Writes tests/golden/medium_hub_centres.txt: oracle counts of single centres
(and hyperedge-profile rows) of the medium workload where the exact counter's
work concentrates.

    python -m oracle.make_medium_hub_golden [--threads N]

Test infrastructure: this script calls only ``oracle/`` (the plain MoCHy-E of
Algorithms 1-2 and the per-hyperedge instance enumeration of section 3.2) and
``workloads/`` (the seeded input generator).  Nothing from the HIP library is
read or run.

Why single centres: Algorithm 2 counts a pair {e_j, e_k} at centre e_i only if
the two are disjoint or i < min(j, k), which attributes every instance to
exactly one centre (section 4.2), so the counts of any centre are a well
defined slice of the total that can be checked on its own.  The medium
workload's rows of line-graph degree above 8,192 hold about 98 % of its
MoCHy-E candidates; the rows picked here are
  * the ten rows of largest line-graph degree (the maximum-degree row first),
  * three rows at evenly spaced ranks within each degree band
    [8192, 12288), [12288, 16384), [16384, 24576), [24576, 32768),
    [32768, max],
and two hyperedge-profile rows (every instance containing the hyperedge,
the work of one MoCHy-A sample) of degree near 8,200 and 16,400.

The file is keyed by the sha256 of the workload's CSR arrays, so a test can
tell a changed generator from a wrong count.
"""
from __future__ import annotations

import argparse
import concurrent.futures
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import native  # noqa: E402
from workloads import make_config  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "medium_hub_centres.txt")
BANDS = [(8192, 12288), (12288, 16384), (16384, 24576), (24576, 32768), (32768, 1 << 30)]
PROFILE_DEGREES = (8200, 16400)


def csr_digest(h) -> str:
    d = hashlib.sha256()
    d.update(np.ascontiguousarray(h.edge_ptr, dtype=np.int64).tobytes())
    d.update(np.ascontiguousarray(h.edge_nodes, dtype=np.int32).tobytes())
    d.update(str(h.num_nodes).encode())
    return d.hexdigest()


def pick_centres(deg: np.ndarray) -> list[int]:
    order = np.argsort(-deg, kind="stable")
    picked = [int(x) for x in order[:10]]
    for lo, hi in BANDS:
        rows = np.nonzero((deg >= lo) & (deg < hi))[0]
        rows = rows[np.argsort(-deg[rows], kind="stable")]
        rows = [int(r) for r in rows if int(r) not in picked]
        if not rows:
            continue
        for q in (0.1, 0.5, 0.9):
            picked.append(rows[min(len(rows) - 1, int(q * len(rows)))])
    return picked


def pick_profile_rows(deg: np.ndarray, exclude) -> list[int]:
    out = []
    for d in PROFILE_DEGREES:
        cand = np.argsort(np.abs(deg - d), kind="stable")
        out.append(next(int(x) for x in cand if int(x) not in exclude and int(x) not in out))
    return out


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    h = make_config("medium")
    digest = csr_digest(h)
    deg, W = native.line_graph_degrees(h, args.threads)
    centres = pick_centres(deg)
    profiles = pick_profile_rows(deg, set(centres))
    jobs = [("exact", c) for c in centres] + [("profile", e) for e in profiles]
    # largest first so the long jobs overlap
    jobs.sort(key=lambda kv: -int(deg[kv[1]]))
    t0 = time.time()

    def run(job):
        kind, x = job
        t = time.time()
        if kind == "exact":
            _, c431, inv = native.mochy_e_centers(h, [x], nthreads=1)
            assert inv == 0
        else:
            _, hp431, inv = native.hyperedge_profiles(h, x, x + 1, nthreads=1)
            assert int(inv[0]) == 0
            c431 = hp431[0]
        print(f"{kind} {x} degree {int(deg[x])}: {time.time() - t:.1f} s "
              f"(elapsed {time.time() - t0:.0f} s)", flush=True)
        return kind, x, c431

    with concurrent.futures.ThreadPoolExecutor(max_workers=args.threads) as ex:
        results = list(ex.map(run, jobs))
    results.sort(key=lambda r: (r[0] != "exact", jobs.index((r[0], r[1]))))
    cand = deg * (deg - 1) // 2
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        f.write("# Oracle counts of single centres of the medium workload (20,000 nodes, 100,000 drawn\n"
                "# hyperedges, sizes 2..25 P(s)~s^-2.5, Zipf(1.0), seed 1, duplicates removed).\n"
                "# Written by oracle/make_medium_hub_golden.py, which calls only oracle/ and workloads/.\n"
                "# exact   <centre> <line-graph degree> <431 3h-motif counts Algorithm 2 attributes to it>\n"
                "# profile <hyperedge> <line-graph degree> <431 counts of the instances containing it>\n"
                f"# candidates of the exact centres: {int(sum(cand[c] for c in centres))} of "
                f"{int(cand.sum())}\n")
        f.write(f"csr_sha256 {digest}\n")
        f.write(f"hyperwedges {W}\n")
        for kind, x, c431 in results:
            f.write(f"{kind} {x} {int(deg[x])} " + " ".join(str(int(v)) for v in c431) + "\n")
    os.replace(tmp, OUT)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
