"""Plain FP64 CPU reference of Bi-cADMM (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls it and shares
no code with it.
"""
from .bicadmm import (BiCADMM, split_columns, prox_squared, prox_logistic, prox_softmax, prox_hinge,
                      zt_step, s_step, topk_support, loss_value, objective)

__all__ = ["BiCADMM", "split_columns", "prox_squared", "prox_logistic", "prox_softmax", "prox_hinge",
           "zt_step", "s_step", "topk_support", "loss_value", "objective"]
