"""Test oracle for the IFGF combined-field apply (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import anything from this package.  The HIP library never calls it and
shares no code, table or helper with it.

Contents
--------
direct      FP64 direct O(N^2) sums of the discrete combined-field operator
            (paper Section 3, eq. field1, with the kernel of Section 2.2),
            in plain C/OpenMP (libdirect.so) and independently in NumPy.
ifgf_ref    A plain NumPy FP64 rendering of the IFGF method of Section 3
            (Algorithm 1) on small inputs, stage by stage, used to check the
            GPU stages array-for-array.  The IFGF value itself is an
            approximation; it is pinned by exact special cases (constant
            kernel, depth <= 2, polynomial reproduction) and by its error
            against `direct`.
"""
