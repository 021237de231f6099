"""FP64 CPU oracle for the PtyRAD multislice hot path.

TEST INFRASTRUCTURE ONLY.  Only `tests/`, `__graft_entry__.smoke()` and the
CPU-baseline leg of `bench.py` may import anything under `oracle/`.  The
product package never imports it, and the oracle never imports the product
package (the seeded input generator `paper_2505_07814_amd.synth` is the single
shared module, and it holds none of the method's arithmetic).
"""
