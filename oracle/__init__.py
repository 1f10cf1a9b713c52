"""CPU oracle for the SMG-preconditioned Krylov solvers (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the GPU library.
"""
