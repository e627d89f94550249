"""FP64 CPU oracle for the conjunctive ML-UDF query (TEST INFRASTRUCTURE ONLY).

This package is the reference the HIP path is checked against.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it; the
product path never does, and it shares no code with the HIP library (only the
seeded input generator ``hydro_synth`` serves both).

What it computes follows the paper (Hydro, arXiv 2403.14902):

* A conjunctive query keeps the tuples on which every UDF predicate holds
  (section 1, the motivating query; section 4.1, the UC1 query).  Predicate
  reordering, short-circuiting and eager dropping of failing rows change only
  the work done, never the answer (section 2.1: Hydro's optimisations do not
  change query accuracy; section 3.3, "Eager Materialization").  The oracle
  therefore evaluates every predicate on every tuple in written order, in FP64,
  and returns the sorted ids of the tuples that pass all of them.
* Routing-policy keys (section 4.1, "Cost-Driven Routing Policy" and "System
  Variants"): score = cost / (1 - selectivity), cost alone, selectivity alone;
  lowest key first.
* Per-predicate statistics under a route (section 3.3, "Metadata for Data
  Routing"; section 4.1 "System Variants": selectivity from counts of filtered
  rows).

See ``hydro_oracle`` for the functions and the passage each one follows.
"""
from .hydro_oracle import *  # noqa: F401,F403
