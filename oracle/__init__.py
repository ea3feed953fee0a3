"""FP64 CPU oracle of the Jump Restore process -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The product path never calls it.
"""
