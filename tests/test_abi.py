"""The C ABI without a GPU: symbols, host-only planning, argument errors.

Plan creation is host-only, so the plan integers (zeta, s_i, L_i, tail) are
compared here with the oracle's own planner, which shares no code with the
library: the two must agree exactly."""

import ctypes
import os
import re

import numpy as np
import pytest

from oracle import compressed, matrix

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

spt = pytest.importorskip("paper_2004_11610_amd")
from paper_2004_11610_amd import _lib  # noqa: E402


def declared_symbols():
    with open(os.path.join(ROOT, "include", "spt.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(spt_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_symbols()
    assert "spt_execute" in names and "spt_precompute" in names
    for name in names:
        assert hasattr(lib, name), name
    assert spt.version().startswith("spt")


FAM_IDS = {"chebyshev_t": matrix.CHEBYSHEV_T, "legendre": matrix.LEGENDRE,
           "jacobi": matrix.JACOBI, "laguerre_fn": matrix.LAGUERRE_FN,
           "hermite_fn": matrix.HERMITE_FN, "sine": matrix.SINE,
           "cos_power": matrix.COS_POWER, "cexp": matrix.CEXP,
           "laguerre_spectral": matrix.LAGUERRE_SPECTRAL}

PLAN_CASES = [("legendre", 256, 1e-12, {}), ("legendre", 4096, 1e-12, {}),
              ("legendre", 16384, 1e-7, {}), ("chebyshev_t", 4096, 1e-12, {}),
              ("chebyshev_t", 1000, 1e-8, {}), ("laguerre_fn", 4096, 1e-12, {}),
              ("hermite_fn", 3000, 1e-7, {}), ("jacobi", 65536, 1e-7, dict(alpha=2.0, beta=3.0)),
              ("legendre", 16384, 1e-10, dict(eps2=1e-4, min_block=20)),
              ("legendre", 777, 1e-9, dict(exact_fft_len=True, eps2=1e-3)),
              ("legendre", 40, 1e-7, {}), ("legendre", 33, 1e-7, {}),
              ("sine", 2000, 1e-8, {}), ("cos_power", 1500, 1e-7, dict(power=3)),
              ("cexp", 3000, 1e-12, {}), ("laguerre_spectral", 501, 1e-10,
                                          dict(eta=2500.0, period=4.0))]


@pytest.mark.parametrize("fam,N,eps,kw", PLAN_CASES)
def test_plan_geometry_matches_oracle(fam, N, eps, kw):
    p = spt.Plan(fam, N, eps, **kw)
    ofam = matrix.MatrixFamily(FAM_IDS[fam], 4, alpha=kw.get("alpha", 0.0),
                               beta=kw.get("beta", 0.0))
    ofam.N = N
    oplan = compressed.Plan(ofam, eps, kw.get("eps2", 1e-2), min_block=kw.get("min_block", 32),
                            round_fft=not kw.get("exact_fft_len", False))
    assert p.blocks() == [b.as_tuple() for b in oplan.blocks]
    info = p.info()
    assert info["tail"] == oplan.tail
    assert info["zeta"] == pytest.approx(oplan.zeta, rel=1e-13)
    assert info["n_blocks"] == len(oplan.blocks)
    # covering: retained ranges and the tail tile [0, N) exactly once
    covered = np.zeros(N, dtype=int)
    covered[: info["tail"]] += 1
    for L, m_off, lo, hi in p.blocks():
        assert (L % 2 == 0 or kw.get("exact_fft_len")) and 0 <= lo < hi <= L
        covered[lo + m_off: hi + m_off] += 1
    assert np.all(covered == 1)


def test_direct_mode_plan():
    p = spt.Plan("legendre", 300, 1e-7, mode=spt.MODE_DIRECT)
    assert p.blocks() == [] and p.info()["tail"] == 300


@pytest.mark.parametrize("args", [
    dict(family=0, N=64, eps=1e-7), dict(family=10, N=64, eps=1e-7),
    dict(family="laguerre_spectral", N=64, eps=1e-7),
    dict(family="laguerre_spectral", N=64, eps=1e-7, eta=10.0),
    dict(family="cexp", N=64, eps=1e-7, nodes=np.linspace(0.1, 0.9, 64)),
    dict(family="cos_power", N=64, eps=1e-7), dict(family="cos_power", N=64, eps=1e-7, power=6),
    dict(family="legendre", N=64, eps=1e-7, trig_conv_q=12),
    dict(family="chebyshev_t", N=64, eps=1e-7, trig_conv_q=65),
    dict(family="sine", N=64, eps=1e-7, trig_conv_q=-1),
    dict(family="legendre", N=1, eps=1e-7), dict(family="legendre", N=64, eps=0.0),
    dict(family="legendre", N=64, eps=1.0), dict(family="legendre", N=64, eps=0.5),
    dict(family="legendre", N=64, eps=1e-7, eps2=1e-8),
    dict(family="jacobi", N=64, eps=1e-7, alpha=-1.0),
    dict(family="legendre", N=64, eps=1e-7, mode=2),
    dict(family="legendre", N=64, eps=1e-7, precisions=8),
    dict(family="legendre", N=64, eps=1e-7, min_block=-1),
    dict(family="legendre", N=64, eps=1e-7, executor=3),
    dict(family="legendre", N=64, eps=1e-7, executor=-1),
])
def test_plan_create_rejects_bad_arguments(args):
    with pytest.raises(spt.SptError) as e:
        spt.Plan(**args)
    assert e.value.code == -1
    assert _lib.load().spt_last_error()


def test_null_and_unprecomputed_calls():
    lib = _lib.load()
    assert lib.spt_plan_create(None, 2, None, 64, 1e-7) == -1
    assert lib.spt_precompute(None, None) == -1
    assert lib.spt_plan_query(None, None) == -1
    assert lib.spt_plan_destroy(None) == 0
    p = spt.Plan("legendre", 64, 1e-7)
    x = ctypes.c_void_p(16)   # never dereferenced: the calls fail before any device work
    y = ctypes.c_void_p(1 << 20)
    assert lib.spt_execute(p.handle, x, y, 1, 0, None) == -2
    assert lib.spt_execute_transposed(p.handle, x, y, 1, 0, None) == -2
    assert lib.spt_plan_nodes(p.handle, (ctypes.c_double * 64)()) == -2
    assert "precomputed" in lib.spt_last_error().decode()
    assert lib.spt_execute_batched(None, None, None, None, 1, 0, None) == -1
    assert lib.spt_execute_batched(None, None, None, None, 0, 0, None) == 0


def test_user_nodes_are_copied():
    nodes = np.linspace(-0.9, 0.9, 50)
    p = spt.Plan("legendre", 50, 1e-7, nodes=nodes)
    assert p.info()["N"] == 50
    with pytest.raises(spt.SptError):
        spt.Plan("legendre", 3, 1e-7, nodes=[0.1, float("nan"), 0.3])


def test_plan_info_layout_matches_header():
    """The binding's spt_plan_info mirrors include/spt.h field by field: the
    header's member names in order equal the ctypes fields, and a plan that is
    not precomputed reports its host-side values with the device-side ones
    (windows, segments) zero."""
    with open(os.path.join(ROOT, "include", "spt.h")) as f:
        text = f.read()
    end = text.index("} spt_plan_info;")
    body = text[text.rindex("typedef struct {", 0, end):end]
    body = re.sub(r"/\*.*?\*/", "", body[body.index("{") + 1:], flags=re.S)
    names = []
    for decl in body.split(";"):
        words = decl.split()
        if not words:
            continue
        # "type a, b[16]": the declarators after the type
        for d in " ".join(words[1:]).split(","):
            names.append(re.sub(r"\[\d+\]", "", d).strip())
    assert names == [f for f, _ in _lib.SptPlanInfo._fields_]
    p = spt.Plan("legendre", 4096, 1e-7)
    info = p.info()
    assert info["N"] == 4096 and info["precomputed"] == 0 and info["n_blocks"] > 0
    assert info["window_lds"] == 0 and info["window_chunked"] == 0
    assert info["transposed_segment"] == 0


def test_exec_wait_bound_arguments():
    lib = _lib.load()
    assert lib.spt_plan_set_exec_wait(None, 0) == -1
    p = spt.Plan("legendre", 64, 1e-7, executor=spt.EXECUTOR_PERSISTENT)
    p.set_exec_wait(1)   # no launch context yet: host state only
    p.set_exec_wait(0)
    with pytest.raises(spt.SptError) as e:
        p.set_exec_wait(-1)
    assert e.value.code == -1


def test_execute_batched_checks_every_tensor():
    """The binding validates each (plan, X, Y) of a batch before any device
    call: dtype, device, shape and output size."""
    import torch
    p = spt.Plan("legendre", 64, 1e-7)
    q = spt.Plan("legendre", 96, 1e-7)
    x = torch.zeros((2, 64), dtype=torch.float64)
    y = torch.zeros((2, 64), dtype=torch.float64)
    with pytest.raises(ValueError):   # host tensors
        spt.execute_batched([p], [x], [y], prec=spt.F64)
    with pytest.raises(ValueError):   # a float64 X for the float32 paths
        spt.execute_batched([p], [x], [y], prec=spt.SPLIT_BF16)
    with pytest.raises(ValueError):   # lengths differ
        spt.execute_batched([p, q], [x], [y], prec=spt.F64)
    with pytest.raises(ValueError):   # missing output
        spt.execute_batched([p], [x], [None], prec=spt.F64)


def test_set_allocator_arguments():
    lib = _lib.load()
    assert lib.spt_set_allocator(_lib.ALLOC_FN(lambda n, s, c: 0), _lib.FREE_FN(), None) == -1
    assert lib.spt_set_allocator(_lib.ALLOC_FN(), _lib.FREE_FN(), None) == 0


@pytest.mark.parametrize("args,code", [
    (dict(family="cexp", N=64, eps=1e-7, mode=3), -5),
    (dict(family="cexp", N=64, eps=1e-7, precisions=1 << 2), -5),
])
def test_complex_plan_refusals(args, code):
    with pytest.raises(spt.SptError) as e:
        spt.Plan(**args)
    assert e.value.code == code


def test_tuning_arguments():
    p = spt.Plan("legendre", 512, 1e-7)
    assert p.tuning() == {"product": 0, "window_rhs": 0, "fft_batch": 0, "fft_half": 0,
                          "inv_four": 0}
    p.set_tuning(product=spt.PRODUCT_CHUNKED, fft_batch=2)   # before precompute: host only
    assert p.tuning()["product"] == 3 and p.tuning()["fft_batch"] == 2
    for bad in (dict(product=5), dict(window_rhs=48), dict(fft_batch=3), dict(fft_half=4)):
        with pytest.raises(spt.SptError) as e:
            p.set_tuning(**bad)
        assert e.value.code == -1
    with pytest.raises(ValueError):
        p.set_tuning(nonsense=1)
    lib = _lib.load()
    assert lib.spt_autotune(p.handle, 4, 0, None, None, None, None) == -2
