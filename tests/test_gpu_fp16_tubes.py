"""FP16-deviation storage on the whole 4096-tube D1Q3 batch for its 1000
steps, against the FP64 form of the same batch, in the configuration the
benchmark times (cached launch shape, HIP graphs of 50 steps rounded to whole
launches).  The FP64 form itself is checked against the oracle elsewhere and
here on every instance whose stability outcome differs.

Bounds and their reasoning (stated before the run): per-instance L2-relative
error of rho <= 0.04 and of u <= 0.2 (2^-12 rms rounding of each stored
deviation per step, accumulating as a random walk over 1000 steps, times an
amplification of 5); max-relative error <= 0.05 (rho) and 0.1 (u) where the
FP64 fronts are resolved (total variation of rho at most 1.2 times the
initial jump), and <= 0.75 (rho) and 1.5 (u) where SRT near tau = 1/2 leaves
grid-scale oscillations behind its fronts, whose displacement by a node or
two the pointwise error then measures.  The stability outcome may differ on
at most 2% of the instances, each of which must either come within 0.1 W_+
rho0 of the criterion in the FP64 oracle before its first unstable step, or
be decided at a step >= n/2, once a wave reflected from an end wall can
exist."""
import multiprocessing as mp
import os

import numpy as np
import pytest

from paper_1801_03863_amd import inputs as I

pytestmark = pytest.mark.gpu

CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1801_03863_amd",
                     "tune_cache_gfx950.txt")
STEPS = 1000


def run_batch(B, torch, tubes, rho, ux, precision):
    params = [B.make_params("d1q3", "srt", "tube", precision, n, 1, tau, 0.0, 0.0, 0.5 * (rl + rr))
              for n, rl, rr, tau in tubes]
    ws = torch.empty(B.lbm_workspace_bytes_batch(params), dtype=torch.uint8, device="cuda")
    ctx = B.lbm_init_batch(params, rho, ux, None, workspace=ws)
    try:
        v = B.lbm_autotune(ctx, CACHE)
        spl = B.lbm_variant_steps(ctx, v)
        B.lbm_set_graph_chunk(ctx, -(-50 // spl) * spl)
        B.lbm_step(ctx, STEPS)
        r, u, _ = B.lbm_moments(ctx)
        st = B.lbm_status_batch(ctx, len(params))
    finally:
        B.lbm_free(ctx)
    return r, u, st


def test_fp16dev_tube_batch_full_length_against_fp64():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1801_03863_amd import binding as B
    tubes = I.tube_batch(count=4096)
    ns = np.array([t[0] for t in tubes])
    pre = np.r_[0, np.cumsum(ns)]
    rho = np.concatenate([I.tube_fields(n, rl, rr)[0] for n, rl, rr, tau in tubes])
    ux = np.zeros_like(rho)
    print("fp16 tubes: FP64 batch", flush=True)
    R, U, s64 = run_batch(B, torch, tubes, rho, ux, "fp64")
    print("fp16 tubes: FP16-deviation batch", flush=True)
    r16, u16, s16 = run_batch(B, torch, tubes, rho, ux, "fp16dev")
    u64 = np.array([s["unstable"] for s in s64])
    uf = np.array([s["unstable"] for s in s16])

    # Stability outcomes: few differences, each explained.
    diff = [int(k) for k in np.where(u64 != uf)[0]]
    print("fp16 tubes: unstable %d (FP64) %d (FP16), %d differ" % (u64.sum(), uf.sum(), len(diff)), flush=True)
    assert len(diff) <= 0.02 * len(tubes)
    from oracle_pool import tube_margin
    with mp.get_context("spawn").Pool(min(16, os.cpu_count() or 1)) as pool:
        margins = pool.map(tube_margin, [(k, STEPS) for k in diff])
    for k, o_unst, o_first, margin in margins:
        n = int(ns[k])
        # the FP64 GPU path against the oracle on this instance
        assert o_unst == u64[k], k
        if o_unst:
            assert o_first == s64[k]["first_step"], (k, o_first, s64[k]["first_step"])
        decided = s64[k]["first_step"] if u64[k] else s16[k]["first_step"]
        near = abs(margin) <= 0.1
        late = decided >= n // 2
        print("  instance %d n=%d margin %.3g decided at %d (%s)" % (k, n, margin, decided,
              "near the criterion" if near else ("after a reflection" if late else "UNEXPLAINED")), flush=True)
        assert near or late, (k, n, margin, decided)

    # Field errors on instances stable in both forms.
    worst = {"l2": [0.0, 0.0], "res": [0.0, 0.0], "unres": [0.0, 0.0]}
    n_res = 0
    for k, (n, rl, rr, tau) in enumerate(tubes):
        if u64[k] or uf[k]:
            continue
        sl = slice(pre[k] + 1, pre[k + 1] - 1)
        Rk, Uk = R[sl], U[sl]
        dr, du = r16[sl] - Rk, u16[sl] - Uk
        l2 = (np.sqrt((dr ** 2).sum() / (Rk ** 2).sum()), np.sqrt((du ** 2).sum() / (Uk ** 2).sum()))
        mx = (np.abs(dr).max() / np.abs(Rk).max(), np.abs(du).max() / np.abs(Uk).max())
        resolved = np.abs(np.diff(Rk)).sum() <= 1.2 * (rl - rr)
        n_res += resolved
        key = "res" if resolved else "unres"
        for j in (0, 1):
            worst["l2"][j] = max(worst["l2"][j], l2[j])
            worst[key][j] = max(worst[key][j], mx[j])
    print("fp16 tubes: L2 rho %.3g u %.3g; max-rel resolved (%d) rho %.3g u %.3g; under-resolved rho %.3g u %.3g"
          % (*worst["l2"], n_res, *worst["res"], *worst["unres"]), flush=True)
    assert worst["l2"][0] <= 0.04 and worst["l2"][1] <= 0.2
    assert worst["res"][0] <= 0.05 and worst["res"][1] <= 0.1
    assert worst["unres"][0] <= 0.75 and worst["unres"][1] <= 1.5
    assert n_res > 0
