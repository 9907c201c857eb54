"""The batched engine's segment-width tuner (sscs_batch_autotune): the
report's shape and choice rule, and solves after tuning against the oracle
(the SpMV's segment width changes only the order of its sums, so every
instance still solves to the tolerance, with the oracle's objective within
1e-6 relative, KKT measures recomputed on the host)."""
import numpy as np
import pytest

from paper_1903_06477_amd import generators as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sscs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_06477_amd import sscs as S
    S.lib()
    return S


def test_autotune_report_and_tuned_solves(sscs):
    import test_gpu_parity as T
    _, S = T._oracle()
    probs = [G.config4_instance(i) for i in range(10)]
    st = T._inexact_settings(sscs)
    bs = sscs.BatchSolver(probs, st)
    _, _, _, before = bs.solve()
    rep = bs.autotune(iters=8)
    print("classes:", [(r["class_seg"], r["chosen_seg"], [round(v, 3) for v in r["ms"]]) for r in rep], flush=True)
    assert len(rep) >= 1
    widths = [r["class_seg"] for r in rep]
    assert widths == sorted(widths) and len(set(widths)) == len(widths)
    for r in rep:
        w0, ms = r["class_seg"], r["ms"]
        assert w0 in (1, 2, 4, 8, 16, 32, 64)
        assert ms[2] > 0.0                          # the rule's own width is always a candidate
        for j, t in enumerate(ms):                  # candidates outside 1..64 are not run
            w = w0 * 2.0 ** (j - 2)
            assert (t < 0) == (w < 1 or w > 64)
        best = min((t, j) for j, t in enumerate(ms) if t >= 0)[1]
        expected = w0 << (best - 2) if best >= 2 else w0 >> (2 - best)
        assert r["chosen_seg"] == expected
    x, y, sv, infos = bs.solve()
    parts = bs.split(x, y, sv)
    for i, p in enumerate(probs[:6]):
        ref = S.solve(p, S.Settings(direction="aa", mem=5, eps=T.EPS_INEXACT, max_iters=20000))
        assert infos[i]["status"] == ref.status == S.SOLVED
        assert max(T.kkt_measures(p, *parts[i])) <= T.EPS_INEXACT * 1.0001
        assert abs(infos[i]["pobj"] - ref.info["pobj"]) <= 1e-6 * (1 + abs(ref.info["pobj"]))
    assert all(inf["status"] == sscs.SOLVED for inf in infos)
    print("iterations before / after tuning:", [b["iters"] for b in before], [a["iters"] for a in infos])
    bs.close()


def test_autotune_rejects_bad_arguments(sscs):
    bs = sscs.BatchSolver([G.config4_instance(0)], sscs.Settings())
    with pytest.raises(sscs.SSCSError):
        bs.autotune(iters=0)
    bs.close()
