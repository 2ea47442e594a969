"""Register and scratch use of the built kernels, from the compiler's
resource remarks that the build collects (paper_2606_26268_amd/_build/
kernel_resources.json; skipped when the library has not been built here).

No kernel spills vector registers or uses scratch memory, except the FP64
LimO3 transport, whose bound of two waves per SIMD makes the compiler spill a
few registers (it runs 31 % faster so than at one wave per SIMD without
spills); and the default kernels keep the occupancy their launch bounds ask
for: four waves per SIMD for the FP32 tiled transport and the implicit
kernels with the network, two for the FP64 LimO3 transport."""
import json
import os

import pytest

PATH = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2606_26268_amd", "_build",
                    "kernel_resources.json")


@pytest.fixture(scope="module")
def res():
    if not os.path.exists(PATH):
        pytest.skip("library not built in this tree")
    return json.load(open(PATH))


# k_transport3d<double, GEOM, true, 8, true>
FP64_LIMO3 = tuple(f"_ZN2m113k_transport3dIdLi{g}ELb1ELi8ELb1EE" for g in range(3))


def test_no_kernel_spills(res):
    bad = {k: v for k, v in res.items()
           if (v.get("scratch", 0) or v.get("vgpr_spill", 0)) and not k.startswith(FP64_LIMO3)}
    assert not bad, bad


def test_fp64_limo3_transport_trades_spills_for_two_waves(res):
    ks = [k for k in res if k.startswith(FP64_LIMO3)]
    assert len(ks) == 3, ks
    for k in ks:
        assert res[k]["waves_per_simd"] >= 2, (k, res[k])
        assert res[k]["vgpr_spill"] <= 32, (k, res[k])


def test_default_kernels_keep_their_occupancy(res):
    # k_transport3d<float, GEOM, false, TY, false> and k_implicit_mlp<R>
    # mangled as ...IfLi<GEOM>ELb<GENERAL>ELi<TY>ELb<LIMO3>...
    fp32_default = [k for k in res if k.startswith("_ZN2m113k_transport3dIfLi")
                    and k.split("ELi")[0].endswith("ELb0") and "ELb0EE" in k.split("ELi")[1]]
    assert len(fp32_default) == 6, fp32_default
    # k_implicit_mlp<R, NT>: both precisions, with and without streaming reads
    mlp = [k for k in res if k.startswith("_ZN2m114k_implicit_mlp")]
    assert len(mlp) == 4, mlp
    for k in fp32_default + mlp:
        assert res[k]["waves_per_simd"] >= 4, (k, res[k])
