"""The paper's physics checks through the HIP path (Sec. 3, Table 1; Sec. 6.1).

The twin-ejecta mock (two homogeneous rest-frame spheres of radius 6 moving
apart along z at Lorentz factor 2, seen at 45 degrees) is rendered by the
batched kernel for routines A (no beaming, no lookback), B (beaming, no
lookback) and C (beaming and lookback), at several observer times and
cadences, and the images are held to the same closed forms the oracle's pins
use: the flux ratios 1, 40.694 (exact for point-symmetric ejecta) and -> 169.27,
the apparent transverse speeds of Eq. 21, the Penrose-Terrell circle, and the
aliasing scale of Eqs. 24-25.  Every image is also compared with the FP64
oracle pixel by pixel (FP64 stacks: 1e-12).
"""
import math

import numpy as np
import pytest

import oracle
import synth
from test_oracle_pins import (EJ, _axis_ratio, _centroid_v, _gap_split, _moments, _row_peaks,
                              _split_flux, alias_case)

pytestmark = pytest.mark.gpu

B = math.sqrt(0.75)
TH = math.pi / 4


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    import paper_2609_09322_amd as d
    return d, torch


def _load(dart, j, b, t):
    return dart.dart_load_epochs(j.shape[1:4][::-1], (1, 1, 1), t, np.ascontiguousarray(j),
                                 np.ascontiguousarray(b), dart.DART_F64)


def _render(dart, torch, st, views):
    imgs = [torch.zeros((v.height, v.width), dtype=torch.float64, device="cuda") for v in views]
    dart.dart_render_batch([st] * len(views), views, imgs)
    return [im.cpu().numpy() for im in imgs]


def _check_oracle(j, b, t, v, img):
    ref, _ = oracle.render(oracle.Stack(j, b, t), oracle.View(v.theta_deg, v.phi_deg, v.width,
                                                             v.height, v.pixel_scale, v.t_obs,
                                                             v.alpha, v.flags & 7))
    floor = 1e-3 * np.abs(ref).max()
    err = (np.abs(img - ref) / np.maximum(np.abs(ref), floor)).max()
    assert err <= 1e-12, err


@pytest.fixture(scope="module")
def ejecta(env):
    dart, torch = env
    times = np.arange(-12.0, 48.0 + 1e-9, 1.0)
    j, b, t = synth.twin_ejecta(dims=EJ["dims"], radius=EJ["radius"], gamma=EJ["gamma"],
                                times=times, t_centre=0.0, sub=4, axis_sep=EJ["axis_sep"])
    return j, b, t, _load(dart, j, b, t)


def test_table1_flux_ratios(env, ejecta):
    dart, torch = env
    j, b, t, st = ejecta
    F64 = dart.DART_F64
    vA = dart.View(45.0, 0.0, 96, 96, 0.5, 0.0, 0.6, dart.DART_NO_LOOKBACK | dart.DART_NO_BEAMING, F64)
    vB = dart.View(45.0, 0.0, 96, 96, 0.5, 0.0, 0.6, dart.DART_NO_LOOKBACK, F64)
    vC = dart.View(45.0, 0.0, 128, 128, 0.4, 0.0, 0.6, 0, F64)
    iA, iB, iC = _render(dart, torch, st, [vA, vB, vC])
    for v, im in ((vA, iA), (vB, iB), (vC, iC)):
        _check_oracle(j, b, t, v, im)
    ua, da = _split_flux(iA, vA, 0.0)
    ub, db = _split_flux(iB, vB, 0.0)
    uc, dc = _split_flux(iC, vC, _gap_split(iC, vC))
    want_b = ((1 + B * math.cos(TH)) / (1 - B * math.cos(TH))) ** 2.6
    print(f"Table 1 on the GPU: A {ua / da:.6f}, B {ub / db:.4f} (40.694), C {uc / dc:.2f} "
          f"(169.27)", flush=True)
    assert ua / da == pytest.approx(1.0, rel=1e-12)
    assert ub / db == pytest.approx(want_b, rel=1e-12)
    assert ub / db == pytest.approx(40.70, abs=0.01)
    assert uc / dc == pytest.approx(oracle.flux_ratio(B, TH, 3.6), rel=0.02)


def test_apparent_speeds_and_penrose_terrell(env, ejecta):
    dart, torch = env
    j, b, t, st = ejecta
    F64 = dart.DART_F64
    nb = dart.DART_NO_BEAMING
    views = [dart.View(45.0, 0.0, 160, 160, 0.4, tt, 0.6, flags | nb, F64)
             for flags in (0, dart.DART_NO_LOOKBACK) for tt in (0.0, 6.0)]
    imgs = _render(dart, torch, st, views)
    _check_oracle(j, b, t, views[0], imgs[0])
    cs = {}
    for k, (v, im) in enumerate(zip(views, imgs)):
        split = _gap_split(im, v) if k < 2 else 0.0
        cs[k] = (_centroid_v(im, v, split, 99), _centroid_v(im, v, -99, split))
    adv = (cs[1][0] - cs[0][0]) / 6.0
    rec = (cs[1][1] - cs[0][1]) / 6.0
    adv0 = (cs[3][0] - cs[2][0]) / 6.0
    print(f"apparent speeds on the GPU: {adv:.4f} / {-rec:.4f} with lookback, {adv0:.4f} without",
          flush=True)
    assert adv == pytest.approx(oracle.apparent_speed(B, TH), rel=0.01)
    assert -rec == pytest.approx(B * math.sin(TH) / (1 + B * math.cos(TH)), rel=0.01)
    assert adv0 == pytest.approx(B * math.sin(TH), rel=0.01)
    # Penrose-Terrell: a circle with lookback, the contracted spheroid without
    assert _axis_ratio(imgs[0], views[0], _gap_split(imgs[0], views[0]), 99) == \
        pytest.approx(1.0, abs=0.05)
    assert _axis_ratio(imgs[2], views[2], 0.0, 99) == pytest.approx(math.sqrt(0.625), abs=0.04)


@pytest.mark.parametrize("dt", [8.0, 4.0, 2.0, 0.5])
def test_aliasing_scale(env, dt):
    dart, torch = env
    j, b, t, ov = alias_case(oracle, dt)
    st = _load(dart, j, b, t)
    v = dart.View(ov.theta_deg, ov.phi_deg, ov.width, ov.height, ov.pixel_scale, ov.t_obs,
                  ov.alpha, dart.DART_NO_BEAMING, dart.DART_F64)
    img = _render(dart, torch, st, [v])[0]
    _check_oracle(j, b, t, v, img)
    r_crit = oracle.alias_r_crit(B, TH, dt)
    R = EJ["radius"]
    sv, su = _moments(img, v)
    peaks = _row_peaks(img)
    print(f"aliasing dt {dt}: R_crit/R {r_crit / R:.2f}, {len(peaks)} peaks, "
          f"sv^2 - su^2 {sv ** 2 - su ** 2:.2f} vs R_crit^2/6 {r_crit ** 2 / 6:.2f}", flush=True)
    if r_crit > 2 * R:
        assert len(peaks) >= 3
    if r_crit < R:
        assert len(peaks) == 1
    if r_crit >= 0.5 * R:
        assert sv ** 2 - su ** 2 == pytest.approx(r_crit ** 2 / 6, rel=0.15)
    else:
        assert sv / su == pytest.approx(1.0, abs=0.03)
