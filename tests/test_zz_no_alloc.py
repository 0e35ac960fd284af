"""af_smooth_eval_static (the no-allocation form of af_smooth_eval, its
scratch in a static device array) against af_smooth_eval through the C ABI:
two calls in a row, the second on a smaller map with fewer pairs, each
bit-identical to af_smooth_eval on the same inputs; a map too large for the
static scratch is refused with AF_ENOMEM."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

C, TS = 0.01, 0.005


def _ctx(synth_mod, w, n_frames):
    import torch
    from paper_2608_06412_amd import Context, default_config
    ctx = Context(default_config(w.voxel, w.trunc, r_c=w.r_c, max_blocks=1 << 15,
                                 max_points=1 << 20))
    for f in w.frames(n_frames):
        ctx.integrate_frame(torch.from_numpy(f.xyz).cuda(), f.origin, f.frame_id)
    return ctx


def _pairs(ctx, w, n, seed):
    rng = np.random.default_rng(seed)
    key = ctx.read_points()["key"]
    from paper_2608_06412_amd.af import unpack_keys
    pts = (unpack_keys(key[rng.choice(len(key), n, replace=True)]) + 0.5) * w.voxel
    p = (pts + rng.uniform(-0.3, 0.3, (n, 3)) * w.voxel).astype(np.float32)
    q = rng.normal(size=(n, 4)).astype(np.float32)
    return p, q


def _eval(ctx, fn, p, q, smp):
    import torch
    n = len(p)
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    s = torch.full((n,), float("nan"), device="cuda")
    dq = torch.full((n, 4), float("nan"), device="cuda")
    dp = torch.full((n, 3), float("nan"), device="cuda")
    getattr(ctx, fn)(cu(p), cu(q), cu(smp), C, TS, s=s, dq=dq, dp=dp)
    torch.cuda.synchronize()
    return s.cpu().numpy(), dq.cpu().numpy(), dp.cpu().numpy()


def test_static_scratch_matches_smooth_eval(synth_mod):
    import torch
    assert torch.cuda.is_available()
    w = synth_mod.tiny()
    smp = synth_mod.tool_samples(synth_mod.cylinder_tool(), 16)
    big = _ctx(synth_mod, w, 20)
    small = _ctx(synth_mod, w, 4)
    assert small.num_blocks() < big.num_blocks()
    cases = [(big, _pairs(big, w, 3000, 1)), (small, _pairs(small, w, 500, 2))]
    for ctx, (p, q) in cases:
        print("map %d blocks, %d pairs" % (ctx.num_blocks(), len(p)), flush=True)
        a = _eval(ctx, "smooth_eval_static", p, q, smp)
        b = _eval(ctx, "smooth_eval", p, q, smp)
        for x, y in zip(a, b):
            assert np.all(np.isfinite(x))
            assert np.array_equal(x.view(np.uint32), y.view(np.uint32))
        assert np.count_nonzero(a[1]) > 0


def test_static_scratch_refuses_a_large_map(synth_mod):
    import torch
    from paper_2608_06412_amd.af import AF_ENOMEM, AFError
    w = synth_mod.tree(n_frames=12)
    ctx = _ctx(synth_mod, w, 12)
    print("tree map: %d blocks" % ctx.num_blocks(), flush=True)
    smp = synth_mod.tool_samples(synth_mod.box_tool(), 16)
    p, q = _pairs(ctx, w, 64, 3)
    with pytest.raises(AFError) as ei:
        _eval(ctx, "smooth_eval_static", p, q, smp)
    assert ei.value.code == AF_ENOMEM
    assert "static scratch" in str(ei.value)
    # the context still evaluates through the allocating form
    s, dq, dp = _eval(ctx, "smooth_eval", p, q, smp)
    assert np.all(np.isfinite(s))
