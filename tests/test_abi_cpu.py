"""Host-side checks of the C ABI: the library loads, exports every symbol
include/itn.h declares, and rejects bad arguments before any launch."""
import os
import re

import numpy as np
import pytest
import torch

import paper_2007_14822_amd as itn
from paper_2007_14822_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "itn.h")).read()
    return sorted(set(re.findall(r"^\s*(?:itn_status|const char\*)\s+(itn_\w+)\s*\(", txt, re.M)))


def test_header_symbols_exported_and_bound():
    lib = L.load()
    syms = _declared_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s
        assert s in L.SIGNATURES, "binding lacks %s" % s
    assert lib.itn_version().decode().startswith("libitn")


@pytest.fixture(scope="module")
def host():
    return itn.Handle(-1)


def _t(*shape, dtype=torch.float64):
    return torch.zeros(*shape, dtype=dtype)


def test_host_handle_refuses_work(host):
    with pytest.raises(itn.ItnError) as e:
        host.contract(_t(2, 3), [1, 2], _t(3, 4), [2, 3], _t(2, 4), [1, 3])
    assert e.value.name == "ITN_E_NODEVICE"


def test_contract_label_errors(host):
    with pytest.raises(itn.ItnError) as e:
        host.contract(_t(2, 3), [1, 2], _t(4, 4), [2, 3], _t(2, 4), [1, 3])
    assert e.value.name == "ITN_E_SHAPE"
    with pytest.raises(itn.ItnError) as e:
        host.contract(_t(2, 3), [1, 2], _t(3, 4), [2, 3], _t(2, 4), [1, 4])
    assert e.value.name == "ITN_E_LABEL"
    with pytest.raises(itn.ItnError) as e:
        host.contract(_t(2, 3), [1, 1], _t(3, 4), [2, 3], _t(2, 4), [1, 3])
    assert e.value.name == "ITN_E_LABEL"
    with pytest.raises(itn.ItnError) as e:
        host.contract(_t(2, 3), [1, 2], _t(3, 4), [2, 3], _t(2, 5), [1, 3])
    assert e.value.name == "ITN_E_SHAPE"


def test_heff_shape_errors(host):
    W = np.zeros((5, 5, 2, 2))
    with pytest.raises(itn.ItnError) as e:  # L not square in its bonds
        host.heff_apply(_t(4, 5, 3), W, W, _t(4, 5, 4), _t(4, 2, 2, 4), _t(4, 2, 2, 4))
    assert e.value.name == "ITN_E_SHAPE"
    with pytest.raises(itn.ItnError) as e:  # W2 with the wrong d
        host.heff_apply(_t(4, 5, 4), W, np.zeros((5, 5, 3, 3)), _t(4, 5, 4), _t(4, 2, 2, 4),
                        _t(4, 2, 2, 4))
    assert e.value.name == "ITN_E_SHAPE"
    with pytest.raises(ValueError):  # W1's d does not fit psi's element count
        host.heff_apply(_t(4, 5, 4), np.zeros((5, 5, 3, 3)), W, _t(4, 5, 4), _t(4, 2, 2, 4),
                        _t(4, 2, 2, 4))
    with pytest.raises(itn.ItnError) as e:  # bf16 psi
        host.heff_apply(_t(4, 5, 4), W, W, _t(4, 5, 4), _t(4, 2, 2, 4, dtype=torch.bfloat16),
                        _t(4, 2, 2, 4))
    assert e.value.name == "ITN_E_DTYPE"
    with pytest.raises(itn.ItnError) as e:  # valid request, no device
        host.heff_apply(_t(4, 5, 4), W, W, _t(4, 5, 4), _t(4, 2, 2, 4), _t(4, 2, 2, 4))
    assert e.value.name == "ITN_E_NODEVICE"


def test_env_update_errors(host):
    W = np.zeros((5, 5, 2, 2))
    with pytest.raises(itn.ItnError) as e:
        host.env_update(_t(3, 5, 3), _t(4, 2, 6), W, "left", _t(6, 5, 6))
    assert e.value.name == "ITN_E_SHAPE"
    with pytest.raises(itn.ItnError) as e:
        host.env_update(_t(3, 5, 3), _t(3, 2, 6), W, "left", _t(6, 5, 5))
    assert e.value.name == "ITN_E_SHAPE"
    with pytest.raises(itn.ItnError) as e:
        host.env_update(_t(3, 5, 3), _t(3, 2, 6), W, "left", _t(6, 5, 6))
    assert e.value.name == "ITN_E_NODEVICE"


def test_workspace_query(host):
    b = host.heff_workspace_size(2048, 2048, 2, 5, 1, "bf16")
    assert b > 2048 * 2048 * 4 * 2


def test_heff_vector_count_and_overlap_checked(host):
    """The binding checks psi / out against nv before the library sees only
    base pointers: a short buffer, a wrong nv and overlapping ranges are
    rejected on the host."""
    W = np.zeros((5, 5, 2, 2))
    L, R = _t(4, 5, 4), _t(4, 5, 4)
    with pytest.raises(ValueError):  # nv = 2 but one vector of psi
        host.heff_apply(L, W, W, R, _t(4, 2, 2, 4), _t(2, 4, 2, 2, 4), nv=2)
    with pytest.raises(ValueError):  # out one element short
        host.heff_apply(L, W, W, R, _t(4, 2, 2, 4), _t(63))
    buf = _t(3, 64)
    with pytest.raises(ValueError):  # out overlaps psi by one vector
        host.heff_apply(L, W, W, R, buf[0:2].reshape(2, 4, 2, 2, 4), buf[1:3].reshape(2, 4, 2, 2, 4),
                        nv=2)
    with pytest.raises(ValueError):
        host.heff_apply_sum([(L, W, W, R)], _t(4, 2, 2, 4), _t(2, 4, 2, 2, 4))


def test_objects_close_and_exit_hook():
    """Handles and plans can be closed explicitly (twice is harmless); open
    ones are registered with the module's exit hook."""
    h2 = itn.Handle(-1)
    h2.close()
    h2.close()
    assert h2.h is None
    with itn.Handle(-1) as h3:
        assert h3.h
    assert h3.h is None
    h4 = itn.Handle(-1)
    assert itn._exit_hook and h4 in itn._live_handles  # the exit hook will close it
    h4.close()


def test_workspace_size_query(host):
    """itn_workspace_size on a host-only handle: the bytes the call would
    take, the call's own validation errors, and no device work."""
    A, B, Cc = _t(40, 30), _t(30, 20), _t(20, 40)
    b_nat = host.workspace_size("contract", A, [1, 2], B, [2, 3], _t(40, 20), [1, 3])
    b_perm = host.workspace_size("contract", A, [1, 2], B, [2, 3], Cc, [3, 1])
    assert b_perm > b_nat > 0  # the permuted output adds a staging buffer
    with pytest.raises(itn.ItnError) as e:
        host.workspace_size("contract", A, [1, 2], B, [2, 3], Cc, [3, 4])
    assert e.value.name == "ITN_E_LABEL"
    W = np.zeros((5, 5, 2, 2))
    hb = host.workspace_size("heff", _t(64, 5, 64), W, W, _t(48, 5, 48), _t(64, 2, 2, 48),
                             prec="bf16")
    hb2 = host.workspace_size("heff", _t(64, 5, 64), W, W, _t(48, 5, 48), _t(2, 64, 2, 2, 48),
                              nv=2, prec="bf16")
    assert hb2 > hb > 64 * 48 * 4 * 2
    eb = host.workspace_size("env", _t(8, 5, 8), _t(8, 2, 12), W, _t(12, 5, 12))
    assert eb > 0
    from oracle import qn as Q
    from paper_2007_14822_amd import inputs as inp
    from tests import qn_util as U
    i = Q.make_index([((0,), 3), ((1,), 2)], +1)
    j = Q.make_index([((0,), 2), ((1,), 4)], +1)
    QA = Q.random_blocks([i, j.dag()], (0,), 1, inp.block_values)
    QB = Q.random_blocks([j, i.dag()], (0,), 2, inp.block_values)
    ref = Q.contract_blocks(QA, [1, 2], QB, [2, 3], [1, 3])
    qb = host.workspace_size("contract", U.desc(QA, with_data=False)[0], [1, 2],
                             U.desc(QB, with_data=False)[0], [2, 3], U.desc(ref, with_data=False)[0],
                             [1, 3])
    assert qb > 0
