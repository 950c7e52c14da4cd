"""Which columns of a batch of NQPs a float32 solve may legitimately take down
a different path than the float64 oracle.

Algorithm 3's coordinate-descent step picks the coordinate with the largest
decrease of the objective.  When the best and the runner-up decrease differ
by less than the rounding error with which a float32 computation knows them,
the float32 solve may pick the other one, and from there its iterate follows
another (equally valid) path: after a few iterations that column can differ
from the oracle's by far more than rounding.  The oracle records every choice
(``oracle.nqp_batch_cdtrace``): the two decreases, the step sizes |delta| of
both, and the size S of the terms its gradient is summed from.  A float32
gradient entry carries an error of about u S (u = 2^-24), so a decrease
m (2g - m) / 2 carries about u S |delta|; a choice is a near-tie when

    best - runner_up < MU * u * S * (|delta_best| + |delta_runner_up|).

MU = 16 leaves room for the gradient's error growing over the incremental
updates of an iteration; on MI355X every flipped column seen had a lead below
6.1 of these units.
"""
import numpy as np

U32 = 2.0 ** -24
MU = 16.0


def near_tied(cd, mu=MU):
    """Boolean per column: does its recorded path contain a near-tie?"""
    ncols = cd.shape[0]
    c = cd.reshape(ncols, -1, cd.shape[-1])
    p, best, sec, db, ds, gs = (c[..., i] for i in range(6))
    valid = (p >= 0) & (sec >= 0)
    noise = U32 * gs * (db + ds)
    return (valid & (best - sec < mu * noise)).any(axis=1)
