"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/mdjk.h, and argument validation fails with the documented
codes before any device work."""
import os
import re

import pytest

from paper_2406_14920_amd import abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mdjk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int|void|const char \*)\s*\**\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = abi.load()
    names = _declared()
    assert "eri_setup" in names and "build_jk" in names and "jk_grad" in names
    for n in names:
        assert hasattr(L, n), n


@pytest.mark.parametrize("shells,xyz,msg", [
    ([(0, 4, [1.0], [1.0])], [[0, 0, 0]], "l=4"),
    ([(0, -1, [1.0], [1.0])], [[0, 0, 0]], "l=-1"),
    ([(0, 1, [], [])], [[0, 0, 0]], "nprim"),
    ([(0, 1, [-1.0], [1.0])], [[0, 0, 0]], "exponent"),
    ([(0, 1, [float("nan")], [1.0])], [[0, 0, 0]], "exponent"),
    ([(0, 1, [1.0], [float("inf")])], [[0, 0, 0]], "coefficient"),
    ([(2, 1, [1.0], [1.0])], [[0, 0, 0]], "atom index"),
    ([(0, 0, [1.0], [1.0])], [[0, float("nan"), 0]], "coordinate"),
])
def test_setup_rejects_bad_input(shells, xyz, msg):
    with pytest.raises(abi.EriError) as e:
        abi.eri_setup(shells, xyz)
    assert e.value.code == abi.ERI_EINVAL
    assert msg in str(e.value)


def test_setup_rejects_bad_options():
    o = abi.eri_default_opts()
    o.schwarz_thresh = -1.0
    with pytest.raises(abi.EriError) as e:
        abi.eri_setup([(0, 0, [1.0], [1.0])], [[0, 0, 0]], o)
    assert e.value.code == abi.ERI_EINVAL
    o = abi.eri_default_opts()
    o.precision = 7
    with pytest.raises(abi.EriError) as e:
        abi.eri_setup([(0, 0, [1.0], [1.0])], [[0, 0, 0]], o)
    assert e.value.code == abi.ERI_EINVAL


def test_null_context_is_a_state_error():
    with pytest.raises(abi.EriError) as e:
        abi.build_jk(0, 1, 2, 3)
    assert e.value.code == abi.ERI_ESTATE
    with pytest.raises(abi.EriError) as e:
        abi.build_jk_static(0, 1, 2, 3)
    assert e.value.code == abi.ERI_ESTATE
    abi.eri_destroy(0)  # NULL is accepted


def test_default_options():
    o = abi.eri_default_opts()
    assert o.schwarz_thresh == 1e-11 and o.prim_thresh == 1e-13
    assert o.precision == abi.ERI_FP64 and o.spherical == 1
