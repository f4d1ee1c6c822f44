"""CPU oracle for the multiobjective perception-aware search.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs anything here; only the test suite, the smoke check and the CPU-baseline
leg of the benchmark do.  The oracle shares no code with the HIP path: the two
meet only at the seeded input generator, which holds none of the method's
arithmetic.

Parts
-----
graph.py    BuildGraph (Alg. 2) and the per-edge/per-node drift inputs
            (Alg. 1 step 2 with the feature-density drift reading), numpy.
mosearch.c  sequential multiobjective label-setting search that returns the
            exact per-node Pareto fronts Alg. 3 is after, plain C.
search.py   ctypes wrapper around mosearch.c.
checks.py   independent references used to pin the search: exhaustive walk
            enumeration, scalar Dijkstra, Bellman-Ford, weighted-sum search.

Every function cites the passage of the paper it follows.
"""
