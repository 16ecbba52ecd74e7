"""The benchmark's throughput metric is Eq. 13 (Mde/s = u_max v_max d_max / t * 1e-6);
pinned against the numbers the paper prints (tests/golden/paper_speed.json)."""
import json
import os

import bench

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_speed.json")


def test_eq13_reproduces_the_printed_throughput():
    g = json.load(open(GOLD))
    t = 1.0 / g["fps"]
    # d_max that makes Eq. 13 reproduce the printed Mde/s at the printed frame rate
    d_max = g["mde_per_s"] * 1e6 * t / (g["u_max"] * g["v_max"])
    assert abs(d_max - 30.0) < 0.01
    assert abs(bench.mde_per_s(g["u_max"], g["v_max"], 30, t) - g["mde_per_s"]) < 0.1


def test_kernel_roofline_units():
    """Cost against HBM at 4 B per distinct cost value (the joint volume), select at
    4 B per entry (the reference volume); the aggregation against the FP32 arithmetic peak at 2m + 2 FLOP per
    entry, m = (2 rho + 1)^2."""
    class P:
        agg_radius = 5
        block_radius = 3
    st = {"cost_volume": 0.1, "aggregate_ref": 0.2, "aggregate_tar": 0.2, "select_subpixel": 0.05}
    k = bench.kernel_rooflines(st, 1280, 720, 64, P)
    n = 1280 * 720 * 64
    # every (d, v) row holds W reference values plus d target values past the right edge
    distinct = sum(720 * (1280 + d) for d in range(64))
    assert k["cost_volume"]["bound"] == "hbm" and k["cost_volume"]["bytes_per_launch"] == 4 * distinct
    assert abs(k["select_subpixel"]["achieved"] - 4 * n / 0.05e-3 / 1e9) < 1.0
    agg = k["aggregate_ref"]
    assert agg["bound"] == "alu" and agg["flops_per_launch"] == (2 * 121 + 2) * n
    assert abs(agg["achieved"] - (2 * 121 + 2) * n / 0.2e-3 / 1e12) < 0.01
    assert abs(agg["frac"] - agg["achieved"] / 157.3) < 1e-3
    # the unfused reference launch also writes its volume
    assert abs(agg["hbm_view"]["achieved_gbs"] - 8 * n / 0.2e-3 / 1e9) < 0.1
    # issued matrix work: 80 x 45 tiles, 4 disparity tiles, 16 patches, 7 K-steps, 3 MFMAs
    # per block: 16 waves x 7 K-steps x (3 MFMAs x 4 disparity tiles + 2 for the weight sums)
    assert agg["mfma_view"]["issued_flops_per_launch"] == 80 * 45 * 16 * 7 * (3 * 4 + 2) * 16384


def test_kernel_sha_covers_every_source():
    for kernel, files in bench.KERNEL_SOURCES.items():
        for f in files:
            assert os.path.exists(os.path.join(bench.CSRC, f)), (kernel, f)
        assert len(bench.kernel_sha(kernel)) == 16


def test_lds_traffic_of_the_tiles():
    """LDS bytes from the tiles' design, counted by hand for 1280x720, D = 64.
    Aggregation, rho = 5: 26 x 28 staged positions; per 16-disparity tile the raw fp32
    tile written and read (2 x 16 x 728 x 4 B), the hi / lo planes (2 x 16 x 728 x 2 B),
    16 waves' B fragments (7 K-steps x 2 planes x 64 lanes x 16 B) and the output tile
    written and read (2 x 16 x 256 x 4 B); per block 56 weights per lane, two 4-byte
    reads each.  Without the direct loads (rho = 6) the raw term is absent."""
    per_tile = 2 * 16 * 728 * 4 + 2 * 16 * 728 * 2 + 16 * 7 * 2 * 64 * 16 + 2 * 16 * 256 * 4
    assert per_tile == 401920
    assert bench.agg_lds_bytes(1280, 720, 64, 5) == 80 * 45 * (4 * per_tile + 1024 * 56 * 2 * 4)
    raw6 = 28 * 28
    tile6 = 2 * 16 * raw6 * 2 + 16 * 8 * 2 * 64 * 16 + 2 * 16 * 256 * 4
    assert bench.agg_lds_bytes(1280, 720, 64, 6) == 80 * 45 * (4 * tile6 + 1024 * 8 * 8 * 2 * 4)
    # cost, r = 2 (direct tile), 21 x 180 blocks of 64 x 4 centres: per entry a window
    # column of 5 and 1/e_r; per block the fills (8 rows of 131 warped + 68 left columns),
    # two row pairs x 127 target centres reading 6 x 5 values and writing 2, 256 left
    # blocks of 25
    per_block = 256 * 64 * 6 + 8 * (131 + 68) + 2 * 127 * (6 * 5 + 2) + 256 * 25
    assert bench.cost_lds_bytes(1280, 720, 64, 2) == 21 * 180 * 4 * per_block
    # cost, r = 3 (sliding-sum tile), 21 x 45 blocks of 64 x 16 centres (22 rows with the
    # halo, 70 left and 133 warped columns, 176 runs of 8 centres, 14 values per run),
    # one chunk of 64 d.  Set-up: left fill, row sums (7 reads, 2 FP64 writes), S_l and
    # 1/e_l (7 x 2 FP64 reads, 12 B written), the runs' left values, 8 waves reading
    # 16 x 64 x 12 B.
    setup = 22 * 70 * 4 + 22 * 64 * (7 * 4 + 16) + 16 * 64 * (7 * 16 + 12) + 176 * 14 * 4 + 8 * 16 * 64 * 12
    assert setup == 303248
    # chunk: warped fill; 127 centres x 4 row groups, 10 rows of 7 reads; 12 B per statistic
    chunk = 22 * 133 * 4 + 127 * 4 * 10 * 7 * 4 + 127 * 16 * 12
    # per disparity: each run reads 14 values and writes 8 sums; each lane reads 22 sums
    # and 16 (S_r, 1/e_r)
    per_d = 176 * (14 * 4 + 8 * 8) + 64 * (22 * 8 + 16 * 12)
    assert bench.cost_lds_bytes(1280, 720, 64, 3) == 21 * 45 * (setup + chunk + 64 * per_d)


def test_kernel_rooflines_with_the_selection_folded_in():
    """With both views aggregated in one launch and the selection folded in, there is
    no select kernel to report: the two-view launch carries both views' FLOPs and reads
    4 B per entry of each view, and the left-right check reads both maps and writes the
    mask, 9 B per pixel."""
    class P:
        agg_radius = 5
        block_radius = 3
    st = {"cost_volume": 0.1, "aggregate_views": 0.45, "lr_check": 0.005}
    k = bench.kernel_rooflines(st, 1280, 720, 64, P, fused=True)
    assert set(k) == {"cost_volume", "aggregate_views", "lr_check"}
    n = 1280 * 720 * 64
    v = k["aggregate_views"]
    assert abs(v["hbm_view"]["achieved_gbs"] - 2 * 4 * n / (0.45e-3) / 1e9) < 0.1
    assert v["flops_per_launch"] == 2 * (2 * 121 + 2) * n
    assert abs(v["achieved"] - 2 * (2 * 121 + 2) * n / (0.45e-3) / 1e12) < 0.01
    assert v["lds_view"]["bytes_per_launch"] == 2 * bench.agg_lds_bytes(1280, 720, 64, 5)
    assert k["lr_check"]["bytes_per_launch"] == 9 * 1280 * 720
    assert abs(bench.agg_stage_ms(st) - 0.455) < 1e-12
    assert abs(bench.agg_stage_ms({"aggregate_ref": 0.25, "aggregate_tar": 0.24}) - 0.49) < 1e-12


def test_adjoint_flop_count_by_hand():
    """adjoint_flops on a 3 x 4 map, window radius 1 (m = 9), block radius 1 (n = 9):
    distinct selected disparities of the Omega pixels in each 3 x 3 window, counted by
    hand."""
    import torch

    class P:
        agg_radius = 1
        block_radius = 1
        D = 8
    d = torch.tensor([[1, 1, 2, 9], [3, 1, 2, 2], [5, 5, 5, 5]], dtype=torch.int32)
    mask = torch.tensor([[1, 1, 1, 1], [1, 0, 1, 1], [0, 0, 0, 1]], dtype=torch.uint8)
    # Omega: (0,0)=1 (0,1)=1 (0,2)=2 (1,0)=3 (1,2)=2 (1,3)=2 (2,3)=5; (0,3) has d = 9 >= D
    # distinct Omega disparities per window (row-major over the 12 pixels)
    per_q = [2, 3, 2, 1, 2, 3, 3, 2, 1, 2, 2, 2]
    fl, n_qd = bench.adjoint_flops(torch, d, mask, P)
    assert n_qd == sum(per_q)
    assert fl == n_qd * 4 * 9 + 7 * 4 * 9 + 12 * 2 * 9
