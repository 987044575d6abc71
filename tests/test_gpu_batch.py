"""Batched advance (many independent 2D grids, one launch per step over a
work list of tiles) checked against single-grid runs of the same problems, bit for bit,
and in FP64 against the oracle. The per-node arithmetic of the two paths is
the same code, so any difference is a bug in the batch bookkeeping (tile
list, offsets, tables, ping-pong) rather than rounding."""
import numpy as np
import pytest

import oracle
import paper_0905_3409_amd as pkg
from gpu_util import TOL64, rel, rel_psi
from paper_0905_3409_amd import inputs

pytestmark = pytest.mark.gpu

# nodes per row straddle the size-class limits 48 / 96 / 192 and are rarely
# multiples of a wave width; one grid is narrower than a 16-wide wave row
SIZES = [(20, 20), (33, 47), (47, 90), (48, 10), (64, 64), (90, 33), (95, 20), (96, 21),
         (130, 200), (191, 9), (192, 9), (260, 75), (12, 140), (300, 300)]


def _workload(sizes=SIZES, seed=11, steps=64, cfl=0.8):
    return inputs.batched_stream_circles(seed=seed, steps=steps, cfl=cfl, sizes=sizes)


def _batch(w, dtype, mixed=pkg.MIXED_CENTRAL, bc=pkg.BC_NEUMANN, widths=None):
    b = pkg.Batch([p["ncell"] for p in w["problems"]], dtype=dtype, mixed=mixed, bc=bc)
    for k, p in enumerate(w["problems"]):
        b.set_velocity(k, w["kind"], p["params"], w["period"])
    if widths is not None:
        b.set_tiles(widths)
    st = b.from_numpy([(p["phi0"], p["psi0"]) for p in w["problems"]])
    return b, st


def _single(p, w, dtype, t0, steps, mixed=pkg.MIXED_CENTRAL, bc=pkg.BC_NEUMANN):
    import torch
    g = pkg.Grid(p["ncell"], dtype=dtype, mixed=mixed, bc=bc, device=0)
    g.set_velocity(w["kind"], p["params"], w["period"])
    st = g.from_numpy(p["phi0"], p["psi0"])
    g.advance(st, t0, w["dt"], steps)
    torch.cuda.synchronize()
    return g.to_numpy(st)


def _assert_same(batch_out, single_out, what):
    for name, a, s in zip(("phi", "psi"), batch_out, single_out):
        bad = np.flatnonzero(~((a == s) | (np.isnan(a) & np.isnan(s))))
        assert bad.size == 0, f"{what}: {name} differs at {bad.size} entries, first {bad[:5]}"


@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("widths", [(64, 64, 64, 64), (32, 32, 32, 32), (16, 16, 16, 16),
                                    (0, 0, 0, 0), (16, 32, 64, 0)])
def test_batch_equals_single_grids_bitwise(dtype, widths):
    import torch
    w = _workload()
    print(f"batch {len(SIZES)} grids {dtype} widths {widths}", flush=True)
    b, st = _batch(w, dtype, widths=widths)
    t0, steps = 0.1, 5  # odd: the result is copied back from the workspace
    b.advance(st, t0, w["dt"], steps)
    torch.cuda.synchronize()
    for k, p in enumerate(w["problems"]):
        _assert_same(b.to_numpy(st, k), _single(p, w, dtype, t0, steps),
                     f"problem {k} {p['ncell']}")


def test_packed_tails_equal_single_grids_bitwise():
    """64-wide waves with ragged columns packed row-major into tiles of their
    own: tails of 1, 3, 47 and 48 columns (packed; 49 and 63 are not), a tail
    over many rows, a grid narrower than a wave, in both precisions."""
    import torch
    sizes = [(2, 2000), (64, 300), (110, 90), (111, 500), (112, 40), (126, 70), (192, 33),
             (46, 5), (200, 7)]
    for dtype in ("float32", "float64"):
        w = _workload(sizes=sizes, seed=18)
        b, st = _batch(w, dtype, widths=(64, 64, 64, 64))
        b.advance(st, 0.05, w["dt"], 3)  # odd: the copy-back kernel's tiles too
        torch.cuda.synchronize()
        for k, p in enumerate(w["problems"]):
            _assert_same(b.to_numpy(st, k), _single(p, w, dtype, 0.05, 3),
                         f"{dtype} problem {k} {p['ncell']}")


@pytest.mark.parametrize("mixed,bc", [(pkg.MIXED_ZERO, pkg.BC_NEUMANN),
                                      (pkg.MIXED_CENTRAL, pkg.BC_EXTRAPOLATE)])
def test_batch_modes_equal_single_grids_bitwise(mixed, bc):
    import torch
    w = _workload(sizes=SIZES[:6] + SIZES[-2:], seed=12, cfl=1.6)
    print(f"batch mixed={mixed} bc={bc}", flush=True)
    b, st = _batch(w, "float32", mixed=mixed, bc=bc, widths=(16, 0, 64, 32))
    b.advance(st, 0.0, w["dt"], 4)
    torch.cuda.synchronize()
    for k, p in enumerate(w["problems"]):
        _assert_same(b.to_numpy(st, k), _single(p, w, "float32", 0.0, 4, mixed, bc),
                     f"problem {k} {p['ncell']}")


@pytest.mark.parametrize("mixed", [pkg.MIXED_CENTRAL, pkg.MIXED_ZERO])
def test_batch_fp64_matches_oracle(mixed):
    import torch
    sizes = [(20, 20), (33, 47), (70, 41), (130, 64), (9, 200)]
    w = _workload(sizes=sizes, seed=13, steps=32, cfl=1.3)
    b, st = _batch(w, "float64", mixed=mixed, widths=(16, 32, 0, 64))
    t0, steps = 0.25, 3
    b.advance(st, t0, w["dt"], steps)
    torch.cuda.synchronize()
    for k, p in enumerate(w["problems"]):
        ncell = p["ncell"]
        o = oracle.advance(2, ncell, (0.0, 0.0), (1.0, 1.0), w["kind"], p["params"], w["period"],
                           p["phi0"], p["psi0"], t0, w["dt"], steps, mixed_mode=mixed)
        g = b.to_numpy(st, k)
        hmin = 1.0 / max(ncell)
        print(f"  {ncell}: phi {rel(g[0], o[0]):.2e} psi/scale "
              f"{rel_psi(g[1], o[1], o[0], hmin):.2e}")
        assert rel(g[0], o[0]) <= TOL64
        assert rel_psi(g[1], o[1], o[0], hmin) <= TOL64


@pytest.mark.parametrize("steps", [6, 5])
def test_graph_replays_equal_direct_launches(steps):
    """The captured advance, replayed several times with eager work and
    synchronisation in between, gives what direct launches give, each time."""
    import torch
    w = _workload(sizes=SIZES[::2], seed=14)
    b, st = _batch(w, "float32", widths=(32, 32, 64, 64))
    direct = st.clone()
    torch.cuda.synchronize()  # the clone reads st on this stream; s then writes it
    s = torch.cuda.Stream()
    for rep in range(3):
        with torch.cuda.stream(s):
            b.advance(st, 0.3, w["dt"], steps, graph=True, stream=s)
        torch.cuda.synchronize()  # both runs share the batch's workspace
        b.advance(direct, 0.3, w["dt"], steps)
        torch.cuda.synchronize()
        junk = torch.ones(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        assert float(junk) == float(1 << 20)
        for k in range(b.nprob):
            _assert_same(b.to_numpy(st, k), b.to_numpy(direct, k), f"replay {rep} problem {k}")


def test_graph_recaptured_after_changes():
    """A change of t0, of the tiles or of a velocity drops the cached graph."""
    import torch
    w = _workload(sizes=SIZES[:5], seed=15)
    b, st = _batch(w, "float32")
    direct = st.clone()
    torch.cuda.synchronize()  # the clone reads st on this stream; s then writes it
    s = torch.cuda.Stream()
    plan = [dict(t0=0.0), dict(t0=0.5), dict(t0=0.5, tiles=(16, 16, 16, 16)),
            dict(t0=0.5, vel=True)]
    for step in plan:
        if "tiles" in step:
            b.set_tiles(step["tiles"])
        if step.get("vel"):
            q = w["problems"][1]["params"].copy()
            q[0::3] *= -1.0  # amplitudes only; (m, n) stay
            b.set_velocity(1, w["kind"], q, w["period"])
        with torch.cuda.stream(s):
            b.advance(st, step["t0"], w["dt"], 3, graph=True, stream=s)
        torch.cuda.synchronize()  # both runs share the batch's workspace
        b.advance(direct, step["t0"], w["dt"], 3)
        torch.cuda.synchronize()
        for k in range(b.nprob):
            _assert_same(b.to_numpy(st, k), b.to_numpy(direct, k), f"{step} problem {k}")


def test_graph_needs_a_stream():
    w = _workload(sizes=SIZES[:2], seed=16)
    b, st = _batch(w, "float32")
    with pytest.raises(pkg.GalsError):
        b.advance(st, 0.0, w["dt"], 2, graph=True, stream=None)


def test_autotune_picks_valid_shapes():
    import torch
    w = _workload(seed=17)
    b, st = _batch(w, "float32")
    scratch = st.clone()
    ms = b.autotune(scratch, w["dt"], steps=3)
    widths = b.get_tiles()
    print(f"autotune {ms:.3f} ms widths {widths}", flush=True)
    assert ms > 0.0 and all(v in (0, 16, 32, 64) for v in widths)
    b.advance(st, 0.0, w["dt"], 2)
    torch.cuda.synchronize()
    for k in (0, 5, len(SIZES) - 1):
        p = w["problems"][k]
        _assert_same(b.to_numpy(st, k), _single(p, w, "float32", 0.0, 2), f"problem {k}")


def test_autotune_choice_is_recorded_for_the_batch_shape(tmp_path, monkeypatch):
    """After an autotune, a new batch of the same shape starts with the tuned
    wave shapes, and the choice is appended to GALS_TUNE_FILE."""
    f = tmp_path / "tune.txt"
    monkeypatch.setenv("GALS_TUNE_FILE", str(f))
    w = _workload(seed=19)
    b, st = _batch(w, "float32")
    b.autotune(st.clone(), w["dt"], steps=2)
    tuned = b.get_tiles()
    again = pkg.Batch([p["ncell"] for p in w["problems"]], dtype="float32")
    assert again.get_tiles() == tuned
    lines = f.read_text().split()
    assert len(lines) == 5 and [int(v) for v in lines[1:]] == tuned


def test_zero_steps_leave_state_untouched():
    import torch
    w = _workload(sizes=SIZES[:3], seed=18)
    b, st = _batch(w, "float32")
    before = st.clone()
    b.advance(st, 0.0, w["dt"], 0)
    torch.cuda.synchronize()
    assert torch.equal(before, st)


def test_full_batched_workload_sampled():
    """512 problems of 32^2 .. 512^2 cells, FP32, in the configuration the
    benchmark times (autotuned wave shapes, graph-captured advance on a side
    stream): sampled problems equal their single-grid runs bit for bit, and an
    FP64 batch of the same problems meets the oracle on the smallest and the
    largest of them."""
    import torch
    w = inputs.batched_stream_circles()
    sizes = [p["ncell"][0] for p in w["problems"]]
    order = np.argsort(sizes, kind="stable")
    sample = sorted({int(order[0]), int(order[1]), int(order[len(order) // 2]),
                     int(order[-1]), 0, 1, 511})
    b, st = _batch(w, "float32")
    scratch = st.clone()
    ms = b.autotune(scratch, w["dt"], steps=2)
    del scratch
    print(f"512 problems, autotune {ms:.3f} ms, widths {b.get_tiles()}", flush=True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.advance(st, 0.0, w["dt"], 3, graph=True, stream=s)
    torch.cuda.synchronize()
    for k in sample:
        p = w["problems"][k]
        print(f"  problem {k} {p['ncell']}", flush=True)
        _assert_same(b.to_numpy(st, k), _single(p, w, "float32", 0.0, 3), f"problem {k}")
    del st, b
    b, st = _batch(w, "float64")
    b.advance(st, 0.0, w["dt"], 2)
    torch.cuda.synchronize()
    for k in (int(order[0]), int(order[-1])):
        p = w["problems"][k]
        o = oracle.advance(2, p["ncell"], (0.0, 0.0), (1.0, 1.0), w["kind"], p["params"],
                           w["period"], p["phi0"], p["psi0"], 0.0, w["dt"], 2)
        g = b.to_numpy(st, k)
        hmin = 1.0 / max(p["ncell"])
        print(f"  FP64 problem {k} {p['ncell']}: phi {rel(g[0], o[0]):.2e} "
              f"psi/scale {rel_psi(g[1], o[1], o[0], hmin):.2e}", flush=True)
        assert rel(g[0], o[0]) <= TOL64
        assert rel_psi(g[1], o[1], o[0], hmin) <= TOL64
