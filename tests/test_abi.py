"""CPU checks of the C ABI: the library loads, exports every entry point that
include/pf.h declares, and rejects bad descriptors and call orders on the host
before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import pf_inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pf_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def pf():
    import paper_1407_8071_amd as pf
    pf.lib()
    return pf


def test_exports_every_declared_symbol(pf):
    names = _declared()
    assert len(names) >= 20
    L = C.CDLL(pf.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def _bytes(pf, specs, ens, options=0):
    models = [pf.PFModel(s) for s in specs]
    md = (pf._ModelDesc * len(models))(*[m.desc for m in models])
    ed = (pf._EnsDesc * len(ens))(*[pf._EnsDesc(*e) for e in ens])
    out = C.c_size_t()
    st = pf.lib().pf_workspace_bytes(md, len(models), ed, len(ens), options, C.byref(out))
    return st, out.value


def test_workspace_bytes_and_validation(pf):
    l63 = pf_inputs.lorenz63()
    st, n = _bytes(pf, [l63], [(0, 4, 256, 0, 1)])
    assert st == 0 and n > 4 * 256 * 3 * 4 * 2
    st2, n2 = _bytes(pf, [l63], [(0, 4, 256, 0, 1), (0, 1, 1 << 20, 0, 2)])
    assert st2 == 0 and n2 > n + (1 << 20) * 3 * 4 * 2
    bad = dict(l63, obs_idx=[0, 7])
    assert _bytes(pf, [bad], [(0, 1, 8, 0, 1)])[0] == 1
    assert "obs_index[1] out of range" in pf.lib().pf_last_error().decode()
    assert _bytes(pf, [l63], [(0, 0, 8, 0, 1)])[0] == 1
    assert _bytes(pf, [l63], [(1, 1, 8, 0, 1)])[0] == 1
    assert _bytes(pf, [l63], [(0, 1, 8, 5, 1)])[0] == 1
    assert _bytes(pf, [dict(l63, obs_var=0.0)], [(0, 1, 8, 0, 1)])[0] == 1
    assert _bytes(pf, [dict(l63, dx=4)], [(0, 1, 8, 0, 1)])[0] == 1
    assert "state_dim 3" in pf.lib().pf_last_error().decode()


def test_learned_flag_validation(pf):
    l63, f20 = pf_inputs.lorenz63(), pf_inputs.fhn(20)
    assert _bytes(pf, [l63], [(0, 1, 8, 1, 1)])[0] == 2        # learned needs FH-N
    st0, n0 = _bytes(pf, [f20], [(0, 2, 16, 0, 1)])
    st1, n1 = _bytes(pf, [f20], [(0, 2, 16, 1, 1)])
    assert st0 == 0 and st1 == 0
    assert n1 >= n0 + 4 * 5762 + 4 * 400                       # parameters + nearest map
    assert _bytes(pf, [pf_inputs.fhn(50)], [(0, 1, 4, 1, 1)])[0] == 2  # J > 48
    assert pf.lib().pf_mlp_nparams(20, 2) == 5634
    assert pf.lib().pf_mlp_nparams(22, 2) == 5762
    assert pf.lib().pf_mlp_nparams(3, 1) == 64 * 3 + 64 + 64 * 64 + 64 + 64 + 1
    assert pf.lib().pf_mlp_nparams(32, 2) == -1
    assert pf.lib().pf_mlp_nparams(20, 5) == -1
    # argument checks happen before any device work
    assert pf.lib().pf_mlp_forward(None, 40, 2, None, 1, None, None) == 1
    assert pf.lib().pf_mlp_forward(None, 20, 2, None, -1, None, None) == 1
    assert pf.lib().pf_mlp_forward(None, 20, 2, None, 0, None, None) == 0
    assert pf.lib().pf_proposal_set(None, 0, None, 5634, None) == 1
    # the allocation-free gradient: NULL buffers, and more rows than its
    # static partial-gradient buffer holds, are refused on the host
    fake = C.c_void_p(0x1000)
    assert pf.lib().pf_mlp_loss_grad_noalloc(None, 22, 2, None, None, 16, None, None, None) == 1
    assert pf.lib().pf_mlp_loss_grad_noalloc(fake, 22, 2, fake, fake, 0, fake, None, None) == 1
    assert pf.lib().pf_mlp_loss_grad_noalloc(fake, 22, 2, fake, fake, 46337, fake, None,
                                             None) == 3
    assert "static buffer holds" in pf.lib().pf_last_error().decode()


def test_resampling_scheme_validation(pf):
    l63 = pf_inputs.lorenz63()
    ok = _bytes(pf, [l63], [(0, 2, 64, 0, 1, 2, 0, 0.5)], options=1)
    assert ok[0] == 0
    # the carried log-weights take M N floats more
    base = _bytes(pf, [l63], [(0, 2, 64, 0, 1)], options=1)[1]
    assert ok[1] >= base + 2 * 64 * 4
    assert _bytes(pf, [l63], [(0, 2, 64, 0, 1, 4, 0, 0.0)], options=1)[0] == 1
    assert "unknown resampling scheme" in pf.lib().pf_last_error().decode()
    assert _bytes(pf, [l63], [(0, 2, 64, 0, 1, 0, 0, 1.5)], options=1)[0] == 1
    assert _bytes(pf, [l63], [(0, 2, 64, 0, 1, 0, 0, -0.1)], options=1)[0] == 1
    assert _bytes(pf, [l63], [(0, 2, 64, 0, 1, 0, 7, 0.0)], options=1)[0] == 1
    # other schemes and the ESS schedule: fused path, N <= 8192 only
    assert _bytes(pf, [l63], [(0, 2, 64, 0, 1, 1, 0, 0.0)], options=0)[0] == 2
    assert _bytes(pf, [l63], [(0, 2, 64, 0, 1, 0, 0, 0.5)], options=0)[0] == 2
    assert _bytes(pf, [l63], [(0, 1, 8193, 0, 1, 3, 0, 0.0)], options=1)[0] == 2
    assert "PF_OPT_FUSED" in pf.lib().pf_last_error().decode()
    # the auxiliary filter: fused, bootstrap transition, no ESS threshold
    assert _bytes(pf, [l63], [(0, 2, 64, 2, 1)], options=1)[0] == 0
    assert _bytes(pf, [l63], [(0, 2, 64, 2, 1)], options=0)[0] == 2
    assert _bytes(pf, [l63], [(0, 2, 64, 2, 1, 0, 0, 0.5)], options=1)[0] == 2
    f20 = pf_inputs.fhn(20)
    assert _bytes(pf, [f20], [(0, 2, 64, 3, 1)], options=1)[0] == 2
    assert _bytes(pf, [l63], [(0, 2, 64, 4, 1)], options=1)[0] == 1
    # the default (multinomial at every interval) runs everywhere
    assert _bytes(pf, [l63], [(0, 1, 8193, 0, 1, 0, 0, 0.0)], options=0)[0] == 0


def test_init_rejects_missing_workspace_and_bad_order(pf):
    l63 = pf.PFModel(pf_inputs.lorenz63())
    md = (pf._ModelDesc * 1)(l63.desc)
    ed = (pf._EnsDesc * 1)(pf._EnsDesc(0, 2, 16, 0, 1))
    ctx = C.c_void_p()
    st = pf.lib().pf_init(md, 1, ed, 1, 0, None, 0, None, C.byref(ctx))
    assert st == 3 and not ctx.value
    st = pf.lib().pf_init(md, 1, ed, 1, 0, C.c_void_p(0x1001), 1 << 30, None, C.byref(ctx))
    assert st == 3
    assert pf.lib().pf_step(None, None, None) == 5
    assert pf.lib().pf_estimate(None, None, None, None, None, None) == 5
    assert pf.lib().pf_status_str(2) == b"unsupported"
