"""Register, scratch and LDS figures of the built kernels (CPU only: the
compiler's resource-usage remarks, recorded by the build next to the library).

The m <= 64 analysis kernels are sized for three workgroups per CU: one
wavefront of each workgroup per SIMD, so three wavefronts per SIMD (at most
168 VGPRs) and three workgroups' LDS within the CU's 160 KiB.  The serving
path batches instances into exactly that many resident workgroups; a kernel
edit that adds registers drops it to two without any error, so the figures
are checked here."""
import json
import os

import pytest

from paper_1310_5954_amd import build as B

LDS_PER_CU = 160 * 1024


def _resources():
    if not os.path.exists(B.RESOURCES):
        pytest.fail("no kernel resource record: build the library first (python -m paper_1310_5954_amd.build)")
    rec = json.load(open(B.RESOURCES))
    if rec["build_id"] != B.source_hash():
        pytest.fail("the kernel resource record is from another build of the sources: rebuild the library")
    return rec["kernels"]


def _analysis(ks, p, m):
    names = [n for n in ks if n.startswith(f"_ZN5letkf10k_analysisILi{p}ELi{m}E")]
    assert len(names) == 1, (p, m, names)
    return ks[names[0]]


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_m64_analysis_fits_three_workgroups_per_cu(p):
    r = _analysis(_resources(), p, 64)
    assert r["waves_per_simd"] >= 3, r
    assert r["vgprs"] + r["agprs"] <= 168, r
    assert 3 * r["lds_bytes"] <= LDS_PER_CU, r
    assert r["scratch_bytes"] == 0 and r["vgpr_spill"] == 0, r


@pytest.mark.parametrize("m", [16, 32])
@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_small_analysis_kernels_do_not_spill(p, m):
    r = _analysis(_resources(), p, m)
    assert r["scratch_bytes"] == 0 and r["vgpr_spill"] == 0, r
    assert r["waves_per_simd"] >= 4, r


def test_no_kernel_spills_vector_registers():
    ks = _resources()
    assert len(ks) > 20
    for name, r in ks.items():
        assert r["vgpr_spill"] == 0, (name, r)
