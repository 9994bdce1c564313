"""Oracle runs of single D1Q3 tubes of the seeded tube batch, for a process
pool started with the 'spawn' method (the workers import only the oracle and
the input recipes, never the GPU library)."""
from oracle import oracle as O
from paper_1801_03863_amd import inputs as I


def tube_margin(args):
    """(index, unstable, first_step, min_post / (rho0 W_+)) of tube k of the
    4096-tube batch after `steps` steps, with rho0 the batch's reference
    density (mean of the two sides)."""
    k, steps = args
    n, rl, rr, tau = I.tube_batch(count=4096)[k]
    rho, ux = I.tube_fields(n, rl, rr)[:2]
    r = O.run(O.D1Q3, O.SRT, O.BC_TUBE, n, 1, tau, rho, ux, steps=steps)
    return k, r["unstable"], r["first_step"], r["min_post"] / (0.5 * (rl + rr) / 6.0)
