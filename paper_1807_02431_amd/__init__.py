"""MI355X-native Generalized Parallel Replica (Gen.ParRep) hot path.

The kernels (gfx950 HIP) sit behind the C ABI of include/gpr.h in libgpr_hip.so; this
package is its Python binding.  Importing the package does not load the library; the
first call that needs it does, and fails loudly if it has not been built.
"""
from .gpr import (BUDGET, NOALLOC_MAX_R, OK, OP_DECORRELATE, OP_DEPHASE, OP_PARALLEL_STEP, PATH_PERSISTENT, PATH_PLAIN,
                  GprError, System, batch_advance, batch_run, exit_vote, fv_plan, fv_plan_noalloc, lib, philox_noise,
                  rhat)

__all__ = ["System", "GprError", "lib", "batch_advance", "batch_run", "OP_DECORRELATE", "OP_DEPHASE",
           "OP_PARALLEL_STEP", "philox_noise", "fv_plan", "fv_plan_noalloc", "rhat",
           "exit_vote", "PATH_PLAIN", "PATH_PERSISTENT", "OK", "BUDGET", "NOALLOC_MAX_R"]
