"""CPU checks of the C ABI: the library loads, exports every declared entry
point, the ctypes struct matches the C layout, and host-side validation
rejects bad configurations before touching a device."""
import ctypes as C
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import synthetic as sy

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nnp.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nnp_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2604_21441_amd import _lib as L
    lib = L.load()
    names = _declared()
    assert "nnp_compute" in names and "nnp_create" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(L.SIGNATURES) == set(names)


def test_status_strings_and_version():
    import paper_2604_21441_amd as P
    assert P.nnp_version().count(".") == 2
    assert "cutoff" in P.nnp_status_string(-3)
    assert P.nnp_status_string(0) == "ok"


def test_config_struct_layout_matches_c():
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    from paper_2604_21441_amd import _lib as L
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "nnp.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(nnp_config), offsetof(nnp_config, rad_shift_host),
         offsetof(nnp_config, widths_host), offsetof(nnp_config, celu_alpha),
         offsetof(nnp_config, ke_coulomb), offsetof(nnp_config, n_members));
  return 0;
}
'''
    tmp = os.path.join("/tmp", f"nnp_layout_{os.getpid()}")
    with open(tmp + ".c", "w") as f:
        f.write(src)
    r = subprocess.run([gcc, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                        "-I", "/opt/rocm/include", tmp + ".c", "-o", tmp], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = [int(v) for v in subprocess.run([tmp], capture_output=True, text=True).stdout.split()]
    S = L.nnp_config
    assert out == [C.sizeof(S), S.rad_shift_host.offset, S.widths_host.offset, S.celu_alpha.offset,
                   S.ke_coulomb.offset, S.n_members.offset]


def test_invalid_configs_rejected_on_host():
    import paper_2604_21441_amd as P
    from paper_2604_21441_amd import _lib as L
    cfg = dict(sy.model_config("water"))
    bad = dict(cfg, widths=(128, 100, 128, 96, 1))
    with pytest.raises(P.NNPError) as e:
        P.nnp_create(bad)
    assert e.value.status == L.NNP_EINVAL and "supported networks" in str(e.value)
    bad = dict(cfg, species=(8, 1))
    with pytest.raises(P.NNPError) as e:
        P.nnp_create(bad)
    assert e.value.status == L.NNP_EINVAL
    bad = dict(cfg, rc_ang=np.float32(6.0))
    with pytest.raises(P.NNPError) as e:
        P.nnp_create(bad)
    assert e.value.status == L.NNP_EINVAL
