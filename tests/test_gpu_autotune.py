"""Autotuning of the batched convolution's tile shapes (GPU): the maps are
bitwise the same for every segment height and workgroup count, and the tuned
plan gives the default plan's results."""
import pytest
import torch

from paper_1310_7114_amd import autotune as T
from paper_1310_7114_amd import synth as S

pytestmark = pytest.mark.gpu


def make_plan(itc, cases):
    plan = itc.BatchPlan([torch.from_numpy(c.img) for c in cases], [c.M for c in cases], [c.sigma for c in cases],
                         [c.iters for c in cases])
    return plan, plan.pack_codebooks([c.w0 for c in cases])


def maps_now(plan):
    plan.maps.zero_()
    plan.precompute()
    torch.cuda.synchronize()
    return plan.maps.clone()


def test_maps_do_not_depend_on_the_tile_shape(gpu_lib):
    cases = S.config3_cases(indices=range(0, 1400, 7))  # 200 silhouettes, every radius class
    plan, _ = make_plan(gpu_lib, cases)
    classes = plan.conv_classes()
    assert len(classes) == 3 and all(c["seg_rows"] == 256 for c in classes)
    ref = maps_now(plan)
    for seg, per in ((64, 0), (128, 1), (512, 0), (4096, 2), (192, 0)):
        for c in classes:
            plan.set_conv_shape(c["key"], seg, min(per, c["max_blocks_per_cu"]))
        assert torch.equal(maps_now(plan), ref), (seg, per)


def test_tuned_plan_gives_the_default_results(gpu_lib, tmp_path):
    cases = S.config3_cases(indices=range(3, 1400, 14))
    plan, w0 = make_plan(gpu_lib, cases)
    n = plan.n

    def run():
        w = torch.empty_like(w0)
        sx = torch.empty(n, dtype=torch.float64, device="cuda")
        d = torch.empty_like(sx)
        done = torch.empty(n, dtype=torch.int32, device="cuda")
        plan.run(w0, w, sx, d, done)
        torch.cuda.synchronize()
        return w, sx, d

    ref = run()
    path = str(tmp_path / "tune.json")
    chosen = T.tune_conv(plan, reps=2, path=path)
    assert set(chosen) == {c["key"] for c in plan.conv_classes()}
    for key, ch in chosen.items():
        assert ch["seg_rows"] in T.SEG_CANDIDATES and not ch["cached"]
    for a, b in zip(run(), ref):
        assert torch.equal(a, b)
    # a second plan of the same layout takes the cached shapes
    plan2, _ = make_plan(gpu_lib, cases)
    again = T.tune_conv(plan2, reps=2, path=path)
    assert all(v["cached"] for v in again.values())
    assert {k: (v["seg_rows"], v["blocks_per_cu"]) for k, v in again.items()} == \
           {k: (v["seg_rows"], v["blocks_per_cu"]) for k, v in chosen.items()}


def test_graph_captured_after_tuning_replays_exactly(gpu_lib, tmp_path):
    """A graph captured after tuning equals eager execution on every replay
    (with eager work and synchronisation between the replays)."""
    cases = S.config3_cases(indices=range(5, 1400, 20))
    plan, w0 = make_plan(gpu_lib, cases)
    n = plan.n
    T.tune_conv(plan, reps=2, path=str(tmp_path / "tune.json"))
    w = torch.empty_like(w0)
    sx = torch.empty(n, dtype=torch.float64, device="cuda")
    d = torch.empty_like(sx)
    done = torch.empty(n, dtype=torch.int32, device="cuda")
    plan.run(w0, w, sx, d, done)
    torch.cuda.synchronize()
    ref = (w.clone(), sx.clone(), d.clone())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.run(w0, w, sx, d, done)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.run(w0, w, sx, d, done)
    for _ in range(3):
        w.zero_()
        d.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(w, ref[0]) and torch.equal(sx, ref[1]) and torch.equal(d, ref[2])


def test_bad_shapes_are_rejected(gpu_lib):
    plan, _ = make_plan(gpu_lib, S.config3_cases(indices=range(4)))
    key = plan.conv_classes()[0]["key"]
    with pytest.raises(gpu_lib.ItcError):
        plan.set_conv_shape(key, 32, 0)
    with pytest.raises(gpu_lib.ItcError):
        plan.set_conv_shape(key, 8192, 0)
    with pytest.raises(gpu_lib.ItcError):
        plan.set_conv_shape(key, 256, 999)
    with pytest.raises(gpu_lib.ItcError):
        plan.set_conv_shape(12345, 256, 0)
