"""Error of the half-precision page form (SH bf16; scale, rotation, opacity
fp16; means fp32; all projection and blending fp32) against FP64 renders of
the same resident set, on a three-level LOD city path:

- against the FP64 render of the decoded half attributes: the arithmetic
  error of the fp32 path alone;
- against the FP64 render of the original fp32 attributes: arithmetic plus
  the quantisation of the attributes.

The resident set is the oracle's, which parity makes equal to the GPU's."""
import math

import numpy as np
import pytest

import oracle
from paper_2506_19415_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _psnr(a, b):
    mse = float(np.mean((np.clip(a, 0, 1) - np.clip(b, 0, 1)) ** 2))
    return float("inf") if mse == 0 else 10 * math.log10(1.0 / mse)


def test_half_form_against_fp64():
    import paper_2506_19415_amd as pkg
    sc = synth.scene_city(0, n=400_000, size=300.0, block=60.0, street=12.0)
    cams = synth.path_city(sc, n_frames=60, width=320, height=180)
    osc_half = oracle.OracleScene(sc, 512, 3, 2.0, 2.0, attr_format=1)
    osc_f32 = oracle.OracleScene(sc, 512, 3, 2.0, 2.0, attr_format=0)
    r = pkg.Renderer(sc, 512, 160, lod_levels=3, img=(320, 180), idbuf=(80, 45), cell=2.0, attr_format=1,
                     lod_radius_px=64.0)
    ovm = oracle.OracleVM(osc_half, 160, (320, 180), (80, 45), lod_radius_px=64.0)
    rows = []
    for k in range(60):
        img, out = r.frame([cams[k]])
        ovm.frame([cams[k]])
        if k % 12 != 11:
            continue
        gpu = img[0].cpu().numpy().astype(np.float64)
        ref_half = ovm.render_fp64(osc_half, [cams[k]])[0]
        ref_f32 = ovm.render_fp64(osc_f32, [cams[k]])[0]
        rows.append((k, _psnr(gpu, ref_half), np.abs(gpu - ref_half).max(), _psnr(gpu, ref_f32),
                     np.abs(gpu - ref_f32).max()))
        print(f"frame {k}: vs fp64(half attrs) PSNR {rows[-1][1]:.1f} dB max {rows[-1][2]:.2e}; "
              f"vs fp64(fp32 attrs) PSNR {rows[-1][3]:.1f} dB max {rows[-1][4]:.2e}", flush=True)
    assert min(x[1] for x in rows) >= 60.0      # fp32 arithmetic
    assert min(x[3] for x in rows) >= 40.0      # plus bf16/fp16 attributes
    r.close()
