"""CPU oracle for the running max-min filter -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library
(``paper_cs_0610046_amd``) never imports it, and the two share no code.

Paper: D. Lemire, "Streaming Maximum-Minimum Filter Using No More than Three
Comparisons per Element".

* :func:`naive` -- the definition (Section 1): max/min over every window
  ``[j, j+w)``, by scanning it (Table 1, "naive").
* :func:`wedge` / :class:`Stream` -- the paper's streaming monotonic-wedge
  algorithm (Section 4, Algorithm 1), with value-comparison counting.
* :func:`filter2d` -- rows first, then columns (Section 1); :func:`naive2d`
  -- the 2-D rectangle definition; :func:`morph2d` -- erosion, dilation,
  opening and closing as compositions of the 2-D filter.
* :func:`batched` / :func:`out_offsets` -- one filter per series of a packed
  buffer (independent series; the per-series call is the 1-D oracle).
* :func:`vhgw`, :func:`gil_kimmel`, :func:`minmax3` -- other exact filters
  the paper reviews (Related Work; the w = 3 proposition), with comparison
  counts: cross-checks of the definition and of the paper's bounds.
* :func:`envelope` / :func:`envelope_batched` -- centered envelopes (windows
  [i-r, i+r] truncated at the ends; the time-warping lower-bound use the
  paper cites in Section 1), from the definition.
* :func:`argnaive` -- the leftmost location of each window's max and min,
  from the definition; :func:`argdeque` -- the same in linear time (the
  arg max/min filter the paper notes comes free with stored locations,
  Section 5; ties: leftmost).

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
(brute force on tiny inputs, numpy/scipy library routines, closed forms,
invariants, hand-built worked examples and the paper's comparison bounds).
"""
from .oracle import (DTYPES, build, load, naive, wedge, Stream, filter2d,
                     naive2d, morph2d, batched, out_offsets, n_out, argnaive, argdeque, envelope,
                     envelope_batched, vhgw, gil_kimmel, minmax3)

__all__ = ["DTYPES", "build", "load", "naive", "wedge", "Stream", "filter2d",
           "naive2d", "morph2d", "batched", "out_offsets", "n_out", "argnaive", "argdeque", "envelope",
           "envelope_batched", "vhgw", "gil_kimmel", "minmax3"]
