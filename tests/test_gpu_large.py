"""The large single-GPU workload at full size: 512 x 512 x 2048 cells, 40
epochs, BF16 storage (171.8 GB resident), jet with Lorentz factor 10 and 12
knots, rendered with FP64 ray parameters and Kahan sums at 1024^2.  The
workload's first four views are checked whole against the snapshot-outer
FP64 oracle on the stored values (two epochs in host memory at a time): total
flux within 1e-6, every pixel within 2e-3, cell-steps within 1e-5; the
storage error (the oracle on the stored values against the oracle on the FP32
source fields, in the same pass) is printed beside.
The same domain cut into two 512 x 512 x 1024 slabs, each loaded and rendered
alone and added into one set of images, sums to the whole render (flux within
1e-6, pixels within 1e-5)."""
import gc
import os
import sys
import types

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_large_bf16_stack_flux(capsys):
    import torch
    import paper_2609_09322_amd as dart
    import synth
    sys.path.insert(0, ROOT)
    import bench
    gc.collect()
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    if free < 190e9:
        pytest.skip(f"needs ~180 GB of free device memory, {free / 1e9:.0f} GB free")
    dims, M, gamma, knots, seed = (512, 512, 2048), 40, 10.0, 12, 5
    st, times = bench.build_stack_incremental(dart, torch, dims, M, seed, gamma, knots,
                                              dart.DART_BF16, chunk_bytes=9 << 30)
    L = synth.diag(dims)
    views = [dart.View(th, ph, 1024, 1024, L / 1024, 0.0, 0.6, dart.DART_FORCE_F64_DDA)
             for th, ph, _ in synth.isotropic_views(256, 1005, sizes=(1024,))[:4]]
    imgs = [torch.zeros((1024, 1024), dtype=torch.float32, device="cuda") for _ in views]
    flux, steps = dart.dart_render_batch([st] * len(views), views, imgs)
    ref, src = bench.streamed_oracle_flux(torch, dims, times, seed, gamma, knots, views,
                                          with_source=True)
    for k, ((img, rflux, rsteps), (simg, sflux, _)) in enumerate(zip(ref, src)):
        got = imgs[k].cpu().numpy().astype(np.float64)
        floor = 1e-3 * np.abs(img).max()
        e = (np.abs(got - img) / np.maximum(np.abs(img), floor)).max()
        sfloor = 1e-3 * np.abs(simg).max()
        se = (np.abs(img - simg) / np.maximum(np.abs(simg), sfloor)).max()
        print(f"large view {k}: flux {flux[k]:.9e} vs {rflux:.9e}, max per-pixel err {e:.3e}, "
              f"steps {steps[k]} vs {rsteps}; storage error: per pixel {se:.3e}, flux "
              f"{abs(rflux / sflux - 1):.3e}", flush=True)
        assert flux[k] == pytest.approx(rflux, rel=1e-6)
        assert e <= 2e-3
        assert abs(int(steps[k]) - rsteps) <= 1e-5 * rsteps
    torch.cuda.synchronize()
    dart.dart_free_epochs(st)
    del st
    gc.collect()
    torch.cuda.empty_cache()
    slabs = bench.render_slabs(types.SimpleNamespace(large_slabs=2, steps=1), dart, torch, dims, M,
                               seed, gamma, knots, views, imgs, flux, steps,
                               torch.cuda.current_stream())
    print(f"slabs: {slabs}", flush=True)
    assert slabs["flux_rel_err_vs_whole"] <= 1e-6
    assert slabs["max_pixel_rel_err_vs_whole"] <= 1e-5
    assert slabs["cell_steps_rel_diff"] <= 1e-5
    gc.collect()
    torch.cuda.empty_cache()
