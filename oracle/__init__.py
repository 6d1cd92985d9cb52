"""CPU oracle -- test infrastructure only.

A plain FP64 CPU implementation of the solver's right-hand side, boundary
conditions, TVD-RK3 stepping and a dense forward-mode adjoint, used to check
the GPU library.  Only tests, the smoke check and the CPU-baseline leg of the
benchmark may import it; the product path never does.
"""
