"""The batched render that allocates nothing (its scratch is the library's
fixed device array) against dart_render_batch, through the C ABI: two calls in
a row, the second with a smaller input, each bit-identical in pixels and
cell-steps and equal in flux up to the order of its FP64 atomic sums; batches beyond the fixed scratch, host images and the plain-kernel
flag are refused without touching the images."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _views(dart, n, seed, dims, sizes):
    L = synth.diag(dims)
    return [dart.View(th, ph, P, P, L / P, 0.0, 0.6, flags)
            for (th, ph, P), flags in zip(synth.isotropic_views(n, seed, sizes=sizes),
                                          [0, dart.DART_NEAREST_EPOCH, 0, dart.DART_NO_LOOKBACK] * n)]


def test_noalloc_equals_batch_twice_then_smaller():
    import torch
    import paper_2609_09322_amd as dart
    dims = (96, 80, 112)
    j, b, times = synth.jet_torch(dims, 12, 31, gamma_spine=4.0, n_knots=4)
    st16 = dart.dart_load_epochs(dims, (1, 1, 1), times, j, b, dart.DART_F16)
    st32 = dart.dart_load_epochs(dims, (1, 1, 1), times, j, b, dart.DART_F32)
    del j, b
    stream = torch.cuda.Stream()
    big = _views(dart, 12, 77, dims, (64, 96, 128, 200))
    small = _views(dart, 3, 78, dims, (48, 64))
    for views in (big, small):
        stacks = [st16 if k % 2 == 0 else st32 for k in range(len(views))]
        a = [torch.full((v.height, v.width), -1.0, dtype=torch.float32, device="cuda") for v in views]
        c = [torch.full_like(x, -2.0) for x in a]
        fa, na = dart.dart_render_batch(stacks, views, a, stream=stream)
        fc, nc = dart.dart_render_batch_noalloc(stacks, views, c, stream=stream)
        torch.cuda.synchronize()
        for k in range(len(views)):
            assert torch.equal(a[k], c[k]), k
        # (flux totals are FP64 atomic sums, equal up to their order)
        assert np.allclose(fa, fc, rtol=1e-12, atol=0)
        assert np.array_equal(na, nc) and int(na.sum()) > 0
        print(f"{len(views)} views: flux {fc.sum():.6e}, cell-steps {int(nc.sum())}", flush=True)


def test_noalloc_refusals():
    import torch
    import paper_2609_09322_amd as dart
    dims = (16, 16, 16)
    j = np.ones((2, 16, 16, 16), dtype=np.float32)
    b = np.zeros((2, 16, 16, 16, 3), dtype=np.float32)
    st = dart.dart_load_epochs(dims, (1, 1, 1), [0.0, 10.0], j, b, dart.DART_F32)
    v = dart.View(30.0, 10.0, 64, 64, 0.5, 5.0, 0.6)
    host = np.full((64, 64), 7.0, dtype=np.float32)
    with pytest.raises(dart.DartError) as ei:
        dart.dart_render_batch_noalloc([st], [v], [host])
    assert ei.value.status == dart.DART_E_INVAL and "device memory" in str(ei.value)
    assert (host == 7.0).all()
    img = torch.full((64, 64), 7.0, dtype=torch.float32, device="cuda")
    vp = dart.View(30.0, 10.0, 64, 64, 0.5, 5.0, 0.6, dart.DART_KERNEL_PLAIN)
    with pytest.raises(dart.DartError):
        dart.dart_render_batch_noalloc([st], [vp], [img])
    # 16 MiB of scratch holds about 2M tiles: 2100 views of 1024^2 do not fit
    n = 2100
    views = [dart.View(30.0, 10.0, 1024, 1024, 0.02, 5.0, 0.6)] * n
    # (distinct one-element slices as the images: refused before anything is
    # enqueued, so nothing is written to them)
    with pytest.raises(dart.DartError) as ei:
        dart.dart_render_batch_noalloc([st] * n, views, [img.view(-1)[k:k + 1] for k in range(n)])
    assert ei.value.status == dart.DART_E_INVAL and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert (img == 7.0).all()
    # and a call that fits still works after the refusals
    f, s = dart.dart_render_batch_noalloc([st], [v], [img])
    ref = torch.zeros_like(img)
    f2, s2 = dart.dart_render_batch([st], [v], [ref])
    torch.cuda.synchronize()
    assert torch.equal(img, ref) and f[0] == pytest.approx(f2[0], rel=1e-12) and s[0] == s2[0]
