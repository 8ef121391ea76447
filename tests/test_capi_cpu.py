"""CPU-side checks of the C ABI: the library loads, exports every symbol
include/ofm.h declares, and its host-only cloud sampler reproduces the
oracle's draw bit for bit (no GPU call is made here)."""
import os
import re

import numpy as np
import pytest

from oracle.sampler import sample_cloud as oracle_cloud
from workloads.configs import MASTER_SEED, cloud_spec

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1705_04374_amd", "libofm.so")


def declared_functions():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(ofm_\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def capi():
    if not os.path.exists(LIB):
        import paper_1705_04374_amd.build as b
        b.build()
    from paper_1705_04374_amd import capi
    return capi


def test_library_exports_every_declared_symbol(capi):
    L = capi.lib()
    decl = declared_functions()
    assert len(decl) >= 16
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(capi.EXPORTS) == sorted(decl)


@pytest.mark.parametrize("cloud", ["cloud2d", "cloud50", "cloud500"])
def test_sampler_bitwise_equal_to_oracle(capi, cloud):
    spec = cloud_spec(cloud)
    for idx in range(3):
        a = capi.ofm_sample_cloud(spec, MASTER_SEED, 1, idx)
        b = oracle_cloud(spec, MASTER_SEED, 1, idx)
        assert np.array_equal(a, b)


def test_sampler_rejects_bad_spec(capi):
    spec = dict(cloud_spec("cloud50"))
    spec["cloud_radius"] = -1.0
    with pytest.raises(capi.OfmError):
        capi.ofm_sample_cloud(spec, 1, 0, 0)
    spec = dict(cloud_spec("cloud50"))
    spec["n_bubbles"] = 100000          # cannot fit: the sampler gives up
    spec["r_median"] = 0.05
    spec["r_sigma"] = 0.0
    with pytest.raises(capi.OfmError) as e:
        capi.ofm_sample_cloud(spec, 1, 0, 0)
    assert e.value.code == capi.OFM_EINFEASIBLE
