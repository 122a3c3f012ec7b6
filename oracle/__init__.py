"""FP64 CPU oracle for the Fourier Disparity Layer hot path.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py.  The GPU library and its Python binding never
import, link or execute anything in this package, and this package imports
nothing from them.
"""
