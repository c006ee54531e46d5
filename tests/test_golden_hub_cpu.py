"""The stored hub-centre counts (tests/golden/medium_hub_centres.txt) belong
to the current medium generator and to the oracle: the CSR digest matches,
the rows are the ones the writing script picks, and the smallest stored
centre is recomputed by the oracle here."""
import numpy as np

from conftest import golden
from oracle import native
from oracle.make_medium_hub_golden import csr_digest, pick_centres, pick_profile_rows
from workloads import make_config


def test_hub_golden_is_current():
    rows = golden("medium_hub_centres.txt")
    head = {r[0]: r[1] for r in rows if r[0] in ("csr_sha256", "hyperwedges")}
    exact = [(int(r[1]), int(r[2]), np.array(r[3:], dtype=np.int64)) for r in rows if r[0] == "exact"]
    prof = [(int(r[1]), int(r[2])) for r in rows if r[0] == "profile"]
    h = make_config("medium")
    assert csr_digest(h) == head["csr_sha256"]
    deg, w = native.line_graph_degrees(h, 8)
    assert w == int(head["hyperwedges"])
    centres = pick_centres(deg)
    assert sorted(c for c, _, _ in exact) == sorted(centres)
    assert all(int(deg[c]) == d for c, d, _ in exact)
    assert sorted(e for e, _ in prof) == sorted(pick_profile_rows(deg, set(centres)))
    c, d, want = min(exact, key=lambda x: x[1])
    _, got, inv = native.mochy_e_centers(h, [c], nthreads=1)
    assert inv == 0 and (got == want).all()
