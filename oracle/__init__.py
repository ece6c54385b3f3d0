"""Plain, slow, serial CPU FP64 oracle for the flat-layer inversion.

TEST INFRASTRUCTURE ONLY. Nothing in the product (the HIP library and its
Python binding) imports, links or calls anything in this package; only the
tests, the smoke check and the CPU-baseline leg of the benchmark do. The
oracle shares no code with the GPU path: it is written from the paper with
NumPy (pocketfft FFTs and LAPACK SVDs as library steps) in float64/complex128.

Modules
-------
model       Green function, the discrete operators of eq. (3)-(5), (7)-(9)
regularize  Tikhonov regularization with a discrepancy-chosen parameter for
            one first-kind system A v = w (Algorithm 2, item 1)
invert      Algorithm 2 end to end: W -> v^ -> v -> u -> xi
forward     data generation: Lippmann-Schwinger solve and the data operator
            (the role of Algorithm 1)
adjoint     hand-derived reverse (VJP) and tangent (JVP) of the inversion map

Parity status of every function is stated in its module header.
"""
