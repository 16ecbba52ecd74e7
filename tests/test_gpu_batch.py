"""GPU tests of the batched form: every output of a batch plan equals the plain
path's output for the same pair bit for bit (the plan runs the same arithmetic),
one pair is also checked directly against the FP64 oracle, and plans can be re-run
and autotuned without changing results."""
import numpy as np
import pytest
import torch

import synth
from oracle import stereo as S
from tests import parity as P

pytestmark = pytest.mark.gpu

PRM = synth.MethodParams(D=0, block_radius=3, agg_radius=5, gamma_d=4.0, gamma_r=0.1)


def _say(msg):
    print(msg, flush=True)


def _cases(shapes, seed0):
    out = []
    for k, (H, W, D) in enumerate(shapes):
        c = synth.small_case(H, W, D, 3, 5, seed0 + k, plane_a=0.07, plane_b=4.0 + k,
                             gamma_d=PRM.gamma_d, gamma_r=PRM.gamma_r)
        out.append(c)
    return out


def _pairs(cases):
    pairs = []
    for c in cases:
        cam = (c.camera.f, c.camera.baseline, c.camera.u0, c.camera.v0)
        pairs.append((torch.from_numpy(c.pair.left).cuda(), torch.from_numpy(c.pair.right).cuda(),
                      c.plane, cam, c.params.D))
    return pairs


def _plain(rsv, pair, D):
    left, right, plane, cam, _ = pair
    prm = rsv.StereoParams(D=D, block_radius=3, agg_radius=5, gamma_d=4.0, gamma_r=0.1)
    return rsv.reconstruct(left, right, plane, cam, prm)


def _same(x, y):
    """Bitwise equality that also matches NaN with NaN."""
    if x.is_floating_point():
        return torch.equal(torch.isnan(x), torch.isnan(y)) and torch.equal(x.nan_to_num(), y.nan_to_num())
    return torch.equal(x, y)


def _check_equal(tag, a, b):
    for k in ("disp_ref", "disp_tar", "disp_sub", "valid", "disp_final", "xyz"):
        assert _same(a[k], b[k]), f"{tag}: {k} differs"
    P.check_subpixel_range(f"{tag} disp_sub", a["disp_sub"].cpu().numpy(), a["disp_ref"].cpu().numpy())


SHAPES = [(37, 150, 31), (70, 201, 64), (52, 141, 40), (24, 70, 8), (96, 128, 17), (45, 64, 1)]


def test_batch_equals_plain_bitwise(rsv_gpu):
    rsv = rsv_gpu
    from paper_1807_07433_amd.batch import BatchPlan
    cases = _cases(SHAPES, 700)
    pairs = _pairs(cases)
    _say(f"[batch] {len(pairs)} uneven pairs: plan + run")
    plan = BatchPlan(pairs, PRM)
    _say(f"  plan {plan.info()}")
    plan.run()
    torch.cuda.synchronize()
    for i, (pair, c) in enumerate(zip(pairs, cases)):
        _say(f"  pair {i}: {c.pair.left.shape} D={c.params.D} vs plain")
        _check_equal(f"pair {i}", plan.outputs[i], _plain(rsv, pair, c.params.D))
    _say("  re-run the same plan")
    first = [{k: v.clone() for k, v in o.items() if v is not None} for o in plan.outputs]
    for o in plan.outputs:
        for v in o.values():
            if v is not None:
                v.zero_()
    plan.run()
    torch.cuda.synchronize()
    for i in range(len(pairs)):
        _check_equal(f"rerun {i}", first[i], plan.outputs[i])
    plan.close()


def test_batch_pair_against_oracle(rsv_gpu):
    from paper_1807_07433_amd.batch import BatchPlan
    cases = _cases([(40, 96, 24), (33, 77, 12)], 800)
    pairs = _pairs(cases)
    _say("[batch] 2 pairs vs the FP64 oracle")
    plan = BatchPlan(pairs, PRM)
    plan.run()
    torch.cuda.synchronize()
    for i, c in enumerate(cases):
        p, prm = c.pair, c.params
        ref = S.reconstruct(p.left, p.right, c.plane.as_tuple(),
                            (c.camera.f, c.camera.baseline, c.camera.u0, c.camera.v0), prm.D,
                            prm.block_radius, prm.agg_radius, prm.gamma_d, prm.gamma_r,
                            prm.lr_threshold, prm.sigma_min)
        o = plan.outputs[i]
        H, W = p.left.shape
        v, u = np.mgrid[0:H, 0:W]
        AL, AR = ref["agg_ref"], ref["agg_tar"]
        dref = o["disp_ref"].cpu().numpy().astype(np.int64)
        dtar = o["disp_tar"].cpu().numpy().astype(np.int64)
        P.check_disparity("batch disp_ref", dref, ref["disp_ref"], AL[dref, v, u], AL.max(0))
        P.check_disparity("batch disp_tar", dtar, ref["disp_tar"], AR[dtar, v, u], AR.max(0))
        agree = dref == ref["disp_ref"]
        inner = agree & (ref["disp_ref"] > 0) & (ref["disp_ref"] < prm.D - 1)
        D = prm.D
        dm = np.clip(ref["disp_ref"] - 1, 0, D - 1)
        dp = np.clip(ref["disp_ref"] + 1, 0, D - 1)
        den = 2 * AL[dm, v, u] + 2 * AL[dp, v, u] - 4 * AL[ref["disp_ref"], v, u]
        P.check_subpixel("batch disp_sub", o["disp_sub"].cpu().numpy(), ref["disp_sub"], inner, den, 1e-6)
    plan.close()


def test_batch_realistic_sizes_equal_plain(rsv_gpu):
    """Five pairs drawn like the 64-pair workload: four of 640x360 and 1280x720 (D 32/64/128)
    and one 1920x1080 pair with D = 128, the largest the workload draws."""
    rsv = rsv_gpu
    from paper_1807_07433_amd.batch import BatchPlan
    cases = synth.batch64_mixed(n_pairs=4, sizes=((360, 640), (720, 1280)))
    cases += synth.batch64_mixed(n_pairs=1, sizes=((1080, 1920),), ds=(128,))
    pairs = _pairs(cases)
    _say(f"[batch] realistic sizes {[c.pair.left.shape + (c.params.D,) for c in cases]}")
    plan = BatchPlan(pairs, PRM)
    # default volume budget (2048 MiB): two slots of at most max(1 GiB, largest volume)
    # instead of every volume, plus 12 B per pixel and the lists
    vols = [4 * c.params.D * c.pair.left.shape[0] * (-(-(c.pair.left.shape[1] + c.params.D - 1) // 64) * 64)
            for c in cases]
    pix = sum(c.pair.left.size for c in cases)
    info = plan.info()
    _say(f"  plan {info}; volumes {sum(vols) / 2**30:.2f} GiB, largest {max(vols) / 2**30:.2f} GiB")
    assert info["workspace_bytes"] <= 2 * max(2**30, max(vols)) + 13 * pix + (64 << 20)
    plan.run()
    torch.cuda.synchronize()
    for i, (pair, c) in enumerate(zip(pairs, cases)):
        _check_equal(f"pair {i}", plan.outputs[i], _plain(rsv, pair, c.params.D))
    plan.close()


@pytest.mark.parametrize("budget", [None, 1])  # default budget: one group; 1 MiB: a group per pair
@pytest.mark.parametrize("r,rho,shapes", [
    (3, 6, [(37, 150, 31), (24, 70, 8)]),             # radius 6: every tile in the persistent kernel
    (1, 2, [(20, 3, 5), (30, 90, 17), (9, 5, 4)])])  # widths below 4 there, the rest in the tile kernels
def test_batch_persistent_path_equals_plain(rsv_gpu, r, rho, shapes, budget):
    rsv = rsv_gpu
    from paper_1807_07433_amd.batch import BatchPlan, default_tuning
    prm = synth.MethodParams(D=0, block_radius=r, agg_radius=rho, gamma_d=PRM.gamma_d, gamma_r=PRM.gamma_r)
    cases = [synth.small_case(H, W, D, r, rho, 960 + k, plane_a=0.07, plane_b=4.0 + k,
                              gamma_d=PRM.gamma_d, gamma_r=PRM.gamma_r)
             for k, (H, W, D) in enumerate(shapes)]
    pairs = _pairs(cases)
    t = default_tuning()
    if budget is not None:
        t.volume_budget_mib = budget
    _say(f"[batch] r={r} rho={rho} shapes {shapes} tuning {t.as_dict()}")
    plan = BatchPlan(pairs, prm, t)
    _say(f"  plan {plan.info()}")
    plan.run()
    torch.cuda.synchronize()
    for i, (pair, c) in enumerate(zip(pairs, cases)):
        left, right, plane, cam, D = pair
        p = rsv.StereoParams(D=D, block_radius=r, agg_radius=rho, gamma_d=PRM.gamma_d, gamma_r=PRM.gamma_r)
        _check_equal(f"pair {i}", plan.outputs[i], rsv.reconstruct(left, right, plane, cam, p))
    plan.close()


# budget (MiB): 0 every volume resident; 1 a group per pair (two slots, two graph
# branches); 8 groups of one or two pairs
@pytest.mark.parametrize("largest_first,tiles,cpc,per_pair,budget",
                         [(0, 1, 0, 0, 0), (1, 4, 2, 0, 0), (1, 3, 1, 0, 2048), (1, 4, -1, 0, 0),
                          (0, 1, -1, 1, 0), (1, 2, 0, 1, 2048), (0, 1, -1, 0, 1), (1, 2, 0, 0, 1),
                          (0, 1, -1, 1, 1), (1, 1, -1, 0, 8)])
def test_tuning_variants_equal_plain(rsv_gpu, largest_first, tiles, cpc, per_pair, budget):
    rsv = rsv_gpu
    from paper_1807_07433_amd.batch import BatchPlan, default_tuning
    cases = _cases(SHAPES[:3], 950)
    pairs = _pairs(cases)
    t = default_tuning()
    t.largest_first, t.cost_tiles_per_item, t.cost_blocks_per_cu = largest_first, tiles, cpc
    t.per_pair_launches = per_pair
    t.volume_budget_mib = budget
    _say(f"[batch] tuning {t.as_dict()}")
    plan = BatchPlan(pairs, PRM, t)
    plan.run()
    torch.cuda.synchronize()
    for i, (pair, c) in enumerate(zip(pairs, cases)):
        _check_equal(f"pair {i}", plan.outputs[i], _plain(rsv, pair, c.params.D))
    plan.close()


def test_autotune_picks_a_shape_and_keeps_results(rsv_gpu):
    rsv = rsv_gpu
    from paper_1807_07433_amd.batch import BatchPlan
    cases = _cases(SHAPES[:4], 900)
    pairs = _pairs(cases)
    _say("[batch] autotune")
    tuning, ms = BatchPlan.autotune(pairs, PRM)
    _say(f"  best {tuning.as_dict()}: {ms:.3f} ms")
    assert ms > 0 and 1 <= tuning.cost_tiles_per_item <= 16
    plan = BatchPlan(pairs, PRM, tuning)
    plan.run()
    torch.cuda.synchronize()
    for i, (pair, c) in enumerate(zip(pairs, cases)):
        _check_equal(f"tuned pair {i}", plan.outputs[i], _plain(rsv, pair, c.params.D))
    plan.close()
