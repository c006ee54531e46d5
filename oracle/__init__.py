"""CPU oracle for MoCHy hypergraph-motif counting (arXiv 2310.15668).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import, call, link or execute anything in
this package.  The product library (``paper_2310_15668_amd``) never does, and
this package never imports the product library: the two share no code.

Contents
--------
patterns   overlap patterns, canonical forms, the 26 h-motif / 431 3h-motif
           id tables, and the k-hyperedge pattern census (sections 2.2, 5.1;
           appendices on k-hyperedge motifs and kh-motifs).
native     brute force over all triples, plain MoCHy-E (Algorithms 1-2),
           MoCHy-A+ hit counts (Algorithm 5), Philox4x32-10, line-graph
           degrees and triangles, in C++ behind ctypes.
cp         significance (Eq. 1), characteristic profile (Eq. 2) and the A+
           rescaling, in float64.

Parity pins: every function here is checked by ``tests/test_oracle_*.py``
against facts the paper states, closed forms, brute force or textbook
identities.  Unpinned: the correspondence of ids with the paper's missing
figure beyond the facts listed in ``patterns``.
"""
