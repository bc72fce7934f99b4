"""MI355X-native IRK stage solver with the block-LDU preconditioner P_LD and
AMG V-cycle subsolves.  The compute path lives in the HIP/C++ library
``libirk.so`` (built from ``csrc/``) behind the C ABI declared in
``include/irk.h``; this package only marshals arguments to it.

Submodules load lazily so that importing ``workloads`` (seeded inputs) does not
load the HIP library.
"""
__all__ = ["binding", "solver", "problems", "tableaux", "workloads", "autograd"]
