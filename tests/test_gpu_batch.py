"""Batched uneven frames with mixed L in one call, hipGraph replay, workspace
chunking, tile-shape invariance and the autotuner (GPU, through the C ABI)."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as wl
from parity_util import compare_omega, oracle_cols, oracle_rows

pytestmark = pytest.mark.gpu

# (W, H, L, N, dtype, dirs): ragged sizes, every real dtype, mixed L and N
MIX = [
    (600, 96, 4, 16, np.float32, "xy"),
    (250, 120, 6, 20, np.float64, "xy"),
    (512, 64, 8, 32, np.float16, "x"),
    (360, 90, 4, 12, np.float32, "y"),
    (300, 48, 6, 32, np.float32, "xy"),
    (270, 100, 5, 14, np.float64, "xy"),
    (700, 56, 5, 15, np.uint8, "xy"),       # radix-7 lengths both ways, 8-bit samples
    (263, 40, 4, 16, np.float32, "xy"),     # prime width: Bluestein
    (700, 40, 7, 20, np.float32, "xy"),     # odd L of the lane-pair lag sums, lines over two blocks
]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def make_batch(bm, torch, flags=False):
    specs, host = [], []
    for k, (W, H, L, N, dt, dirs) in enumerate(MIX):
        img = wl.random_frame(W, H, seed=100 + k, dtype=dt, snr_db=6.0 + 2 * k)
        d = torch.from_numpy(img).to("cuda")
        wx = torch.full((H, W), -7.0, device="cuda") if "x" in dirs else None
        wy = torch.full((H, W), -7.0, device="cuda") if "y" in dirs else None
        fl = torch.full((H, W), 255, dtype=torch.uint8, device="cuda") if flags else None
        code = (bm.BM_DIR_X if "x" in dirs else 0) | (bm.BM_DIR_Y if "y" in dirs else 0)
        specs.append(bm.FrameSpec(d, L, N, code, wx, wy, fl))
        host.append(img)
    return specs, host


def outputs(torch, specs):
    torch.cuda.synchronize()
    out = []
    for s in specs:
        for t in (s.omega_x, s.omega_y, s.flags):
            out.append(None if t is None else t.cpu().numpy().copy())
    return out


def same(a, b):
    for u, v in zip(a, b):
        assert (u is None) == (v is None)
        if u is not None:
            assert np.array_equal(u, v, equal_nan=True) if u.dtype.kind == "f" else np.array_equal(u, v)


def test_mixed_batch_matches_single_frame_calls_and_oracle(bm, torch):
    d = bm.Demodulator(0, max_width=1024, max_height=1024, max_batch_pixels=4 << 20)
    specs, host = make_batch(bm, torch)
    bm.bosmusic_demodulate(d.h, specs)
    batched = outputs(torch, specs)
    for s in specs:                       # one frame per call
        bm.bosmusic_demodulate(d.h, [s])
    single = outputs(torch, specs)
    same(batched, single)
    for (W, H, L, N, dt, dirs), img, s in zip(MIX, host, specs):
        if "x" in dirs:
            rows = list(range(0, H, 7))
            compare_omega(s.omega_x.cpu().numpy()[rows], oracle_rows(img, rows, L, N), f"batch x {W}x{H}")
        if "y" in dirs:
            cols = list(range(1, W, 23))
            compare_omega(s.omega_y.cpu().numpy()[:, cols].T, oracle_cols(img, cols, L, N), f"batch y {W}x{H}")
    d.close()


def test_workspace_chunking_gives_identical_results(bm, torch):
    big = bm.Demodulator(0, max_width=1024, max_height=1024, max_batch_pixels=4 << 20)
    small = bm.Demodulator(0, max_width=700, max_height=120)   # about one frame per group
    specs, _ = make_batch(bm, torch)
    bm.bosmusic_demodulate(big.h, specs)
    a = outputs(torch, specs)
    bm.bosmusic_demodulate(small.h, specs)
    b = outputs(torch, specs)
    same(a, b)
    big.close()
    small.close()


def test_pipelined_halves_on_a_side_stream(bm, torch):
    """A batch of two or more frames runs as two halves on two streams; the call stays
    ordered on the caller's stream: work enqueued on it before the call (poisoned
    outputs) is seen, back-to-back calls without a host wait give the single-frame
    results, and the caller's stream holds the finished maps when the call returns."""
    d = bm.Demodulator(0, max_width=1024, max_height=1024, max_batch_pixels=4 << 20)
    specs, _ = make_batch(bm, torch, flags=True)
    for s in specs:
        bm.bosmusic_demodulate(d.h, [s])
    ref = outputs(torch, specs)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        for rep in range(3):
            for s in specs:
                for t in (s.omega_x, s.omega_y):
                    if t is not None:
                        t.fill_(123.0 + rep)
                s.flags.fill_(7)
            bm.bosmusic_demodulate(d.h, specs, stream=side)
            bm.bosmusic_demodulate(d.h, specs[::-1], stream=side)
        snap = [None if t is None else t.clone() for s in specs for t in (s.omega_x, s.omega_y, s.flags)]
    side.synchronize()
    same(ref, [None if t is None else t.cpu().numpy() for t in snap])
    d.close()


def test_graph_replays_match_eager(bm, torch):
    eager = bm.Demodulator(0, max_width=1024, max_height=1024, max_batch_pixels=4 << 20)
    graph = bm.Demodulator(0, max_width=1024, max_height=1024, max_batch_pixels=4 << 20, graph=True)
    specs, _ = make_batch(bm, torch)
    bm.bosmusic_demodulate(eager.h, specs)
    ref = outputs(torch, specs)
    x = torch.randn(1 << 20, device="cuda")
    for rep in range(4):
        for s in specs:                   # poison the outputs between replays
            for t in (s.omega_x, s.omega_y):
                if t is not None:
                    t.fill_(123.0)
        y = (x * 2.0).sum()               # the program's own eager work in between
        bm.bosmusic_demodulate(graph.h, specs)
        torch.cuda.synchronize()
        assert torch.isfinite(y)
        same(ref, outputs(torch, specs))
    eager.close()
    graph.close()


def test_flags_with_both_directions_in_a_batch(bm, torch):
    d = bm.Demodulator(0, max_width=1024, max_height=1024, max_batch_pixels=4 << 20)
    specs, _ = make_batch(bm, torch, flags=True)
    bm.bosmusic_demodulate(d.h, specs)
    torch.cuda.synchronize()
    for s in specs:
        fl = s.flags.cpu().numpy()
        if s.omega_x is not None:
            assert np.array_equal((fl & 1) != 0, np.isnan(s.omega_x.cpu().numpy()))
        else:
            assert np.all((fl & 15) == 0)
        if s.omega_y is not None:
            assert np.array_equal((fl & 16) != 0, np.isnan(s.omega_y.cpu().numpy()))
        else:
            assert np.all((fl & 240) == 0)
    d.close()


def test_tile_shapes_do_not_change_results(bm, torch, tmp_path):
    """Block sizes and grid shapes (one block per item, or a persistent grid) give
    identical results."""
    cache = tmp_path / "tune.jsonl"
    specs, _ = make_batch(bm, torch)
    base = bm.Demodulator(0, max_width=1024, max_height=1024, max_batch_pixels=4 << 20)
    bm.bosmusic_demodulate(base.h, specs)
    ref = outputs(torch, specs)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    for block, gpc in [(128, 0), (128, 1), (256, 2), (256, 16)]:
        with open(cache, "w") as f:
            for (W, H, L, N, dt, dirs) in MIX:
                f.write(json.dumps({"arch": arch, "L": L, "N": N, "block": block, "grid_per_cu": gpc, "us": 1.0},
                                   separators=(",", ":")) + "\n")
        t = bm.Demodulator(0, max_width=1024, max_height=1024, max_batch_pixels=4 << 20, tune_cache=str(cache))
        bm.bosmusic_demodulate(t.h, specs)
        same(ref, outputs(torch, specs))
        t.close()
    base.close()


def test_autotune_picks_a_candidate_and_caches_it(bm, torch, tmp_path):
    cache = tmp_path / "tune.jsonl"
    d = bm.Demodulator(0, max_width=1024, max_height=1024, tune_cache=str(cache))
    us = d.autotune(6, 32, width=1024, lines=256)
    assert us > 0
    line = json.loads(open(cache).read().strip().splitlines()[-1])
    assert line["L"] == 6 and line["N"] == 32 and line["block"] in (128, 256)
    print("autotune", line)
    # a tuned handle still matches the oracle
    img = wl.random_frame(600, 64, seed=3)
    wx, wy = d.demodulate(torch.from_numpy(img).to("cuda"), 6, 32, "xy")
    torch.cuda.synchronize()
    ox, oy = oracle.demodulate(img, 6, 32, "xy")
    compare_omega(wx.cpu().numpy(), ox, "tuned x")
    compare_omega(wy.cpu().numpy(), oy, "tuned y")
    d.close()


def test_every_analytic_kernel_variant_in_one_batch(bm, torch):
    """One call whose line lengths need all four analytic kernel variants (radices up to 5 or
    up to 13, twiddles in LDS or not) plus Bluestein: each frame equals its own single call
    bit for bit and the oracle on sampled lines."""
    shapes = [
        (1024, 6, 6, 20, np.float32),     # radix 4: pairs, twiddles in LDS
        (700, 5, 5, 15, np.uint8),        # radix 7: the large-radix kernel
        (1850, 4, 7, 15, np.float32),     # Bluestein at m = 3750 (5-smooth)
        (8192, 3, 6, 24, np.float32),     # single lines, twiddles in global memory
        (7000, 3, 4, 16, np.float64),     # radix 7, single lines, twiddles in global memory
    ]
    d = bm.Demodulator(0, max_width=8192, max_height=16)
    specs, imgs = [], []
    for k, (W, H, L, N, dt) in enumerate(shapes):
        img = wl.random_frame(W, H, seed=500 + k, dtype=dt, snr_db=8.0)
        specs.append(bm.FrameSpec(torch.from_numpy(img).to("cuda"), L, N, bm.BM_DIR_X,
                                  torch.full((H, W), -7.0, device="cuda")))
        imgs.append(img)
    bm.bosmusic_demodulate(d.h, specs)
    got = outputs(torch, specs)
    for k, (W, H, L, N, dt) in enumerate(shapes):
        single, _ = d.demodulate(specs[k].data, L, N, "x")
        torch.cuda.synchronize()
        assert np.array_equal(got[3 * k], single.cpu().numpy(), equal_nan=True), shapes[k]
        rows = [0, H - 1]
        compare_omega(got[3 * k][rows], oracle_rows(imgs[k], rows, L, N), f"variant batch {W}")
    d.close()


def test_cfg3_full_batch_one_graph_replay_sampled(bm, torch):
    """The whole uneven batch (64 frames, 512x512 .. 2048x1536, L = 4, 6, 8, N = 2L + 8) in
    one cached hipGraph, replayed: sampled rows and columns of every 21st frame against the
    oracle, and the replay equal to the first launch bit for bit."""
    from parity_util import compare_omega, oracle_cols, oracle_rows
    frames = [wl.cfg3_frame(k) for k in range(64)]
    px = sum(f.width * f.height for f in frames)
    d = bm.Demodulator(0, max_width=2048, max_height=1536, graph=True, max_batch_pixels=px)
    imgs = [torch.from_numpy(f.data).cuda() for f in frames]
    outs = [(torch.empty(i.shape, device="cuda"), torch.empty(i.shape, device="cuda")) for i in imgs]
    specs = [bm.FrameSpec(i, f.L, f.N, 3, o[0], o[1]) for i, f, o in zip(imgs, frames, outs)]
    bm.bosmusic_demodulate(d.h, specs)             # capture and first launch
    torch.cuda.synchronize()
    first = [(a.clone(), b.clone()) for a, b in outs]
    for a, b in outs:
        a.fill_(3.0)
        b.fill_(3.0)
    bm.bosmusic_demodulate(d.h, specs)             # replay
    torch.cuda.synchronize()
    for (a, b), (fa, fb) in zip(outs, first):
        assert torch.equal(torch.nan_to_num(a, 9.0), torch.nan_to_num(fa, 9.0))
        assert torch.equal(torch.nan_to_num(b, 9.0), torch.nan_to_num(fb, 9.0))
    for k in (0, 21, 42, 63):
        f = frames[k]
        gx, gy = outs[k][0].cpu().numpy(), outs[k][1].cpu().numpy()
        rows = list(range(5, f.height, f.height // 3))
        cols = list(range(9, f.width, f.width // 3))
        compare_omega(gx[rows], oracle_rows(f.data, rows, f.L, f.N), f"cfg3 graph k{k} x")
        compare_omega(gy[:, cols].T, oracle_cols(f.data, cols, f.L, f.N), f"cfg3 graph k{k} y")
    d.close()
