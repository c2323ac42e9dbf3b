"""CPU reference code for tests and the benchmark's CPU legs -- test
infrastructure only; the product path never imports this package.

* ``cv_oracle``  -- the FP64 oracle: the paper's naive baseline definition.
* ``fast_cpu``   -- the paper's fast algorithm on the CPU in FP64 NumPy, used
                    as a timing baseline and a second cross-check.
"""
