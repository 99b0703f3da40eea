"""The C-ABI library loads and exports every symbol the header declares, and its
host-side logic (status strings, argument checks, sizes) works without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "riccsd.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ri_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_all_declared_symbols():
    from paper_1810_08142_amd import _lib
    L = _lib.lib()
    names = _declared()
    assert names, "no declarations found"
    for n in names:
        assert hasattr(L, n), n
    # the binding covers the same set
    assert set(_lib.declared_symbols()) == set(names)


def test_status_strings_and_flops():
    from paper_1810_08142_amd import _lib
    L = _lib.lib()
    assert L.ri_status_str(0) == b"ok"
    assert L.ri_status_str(2) == b"output overlaps an input"
    # Naux v^3 (v+1) + 2 [p_v^2 p_o + p_v-^2 p_o-] at the c2 sizes
    o, v, n = 16, 256, 768
    pv, pvm, po, pom = v * (v + 1) // 2, v * (v - 1) // 2, o * (o + 1) // 2, o * (o - 1) // 2
    assert L.ri_ppl_flops(o, v, n) == float(n * v**3 * (v + 1) + 2 * (pv * pv * po + pvm * pvm * pom))
    assert L.ri_ppl_flops(0, v, n) == 0.0


def test_argument_checks_before_any_device_work():
    from paper_1810_08142_amd import _lib
    L = _lib.lib()
    assert L.ri_ppl(None, None, 2, 3, 4, None, None) == 1
    assert b"null" in L.ri_last_error_msg()
    assert L.ri_ppl(8, 16, 0, 3, 4, 24, None) == 1
    assert L.ri_ppl_ex(8, 16, 2, 3, 4, 24, 9, None, 0, None) == 1
    assert L.ri_ppl_workspace_bytes(0, 3, 4, 0) == 0
    assert L.ri_ppl_workspace_bytes(2, 20, 8, 0) > 0
    # overlapping output and input
    assert L.ri_ppl(4096, 8192, 2, 3, 4, 8192, None) == 2
    # the split path's size limit: vp * Qp < 2^27
    assert L.ri_ppl_workspace_bytes(2, 8192, 16384, 2) == 0
    assert L.ri_ppl_workspace_bytes(2, 4096, 16384, 2) > 0


def test_mlp_training_options_and_checks():
    from paper_1810_08142_amd import _lib
    L = _lib.lib()
    o = _lib.RIMlpTrainOpts()
    L.ri_mlp_default_train_opts(ctypes.byref(o))
    assert (o.epochs, o.batch, o.shuffle, o.seed) == (30, 4096, 1, 1)
    assert o.lr == pytest.approx(5e-4) and o.warmup == pytest.approx(0.05)
    assert ctypes.sizeof(o) == 40  # int, long, float, float, u64, int (LP64 padding)
    assert L.ri_mlp_train(None, 8, 16, 10, None, None, 0, None, None, None, None) == 1
    assert b"null network" in L.ri_last_error_msg()
    assert L.ri_mlp_init(None, 3, None) == 1
    r = (ctypes.c_double * 2)()
    assert L.ri_tau_pair_asymmetry(None, 2, 3, r, None) == 1
    assert L.ri_tau_pair_asymmetry(64, 0, 3, r, None) == 1


def test_triples_argument_checks():
    from paper_1810_08142_amd import _lib
    L = _lib.lib()
    e = ctypes.c_double()
    assert L.ri_ccsd_triples(None, 8, 8, ctypes.byref(e), None) == 1
    assert L.ri_ccsd_triples_flops(2, 3) == 2 * 3 * 4 * (2.0 * 81 + 2.0 * 27 * 2)
    assert L.ri_ccsd_triples_flops(0, 3) == 0.0


def test_exchange_symmetric_form_flops_and_argument_checks(monkeypatch):
    from paper_1810_08142_amd import _lib
    L = _lib.lib()
    assert L.ri_ppl_sym(None, None, 2, 3, 4, None, None) == 1
    assert L.ri_ppl_sym(8, 16, 0, 3, 4, 24, None) == 1
    assert L.ri_ppl_sym(4096, 8192, 2, 3, 4, 8192, None) == 2
    assert L.ri_ppl_sym_flops(0, 3, 4) == 0.0
    # one slab: nothing is built twice or skipped, the FLOP are those of ri_ppl
    monkeypatch.setenv("RI_PPL_SYM_SLABS", "1")
    assert L.ri_ppl_sym_flops(3, 40, 50) == L.ri_ppl_flops(3, 40, 50)
    # n slabs at o=16 v=256 naux=768: the build falls to about (1 + 1/n)/2, the
    # contraction is unchanged
    o, v, n = 16, 256, 768
    build = float(n * v**3 * (v + 1))
    contract = L.ri_ppl_flops(o, v, n) - build
    for slabs in (2, 8, 136):
        monkeypatch.setenv("RI_PPL_SYM_SLABS", str(slabs))
        got = L.ri_ppl_sym_flops(o, v, n) - contract
        assert build / 2 < got <= build * (1 + 1 / slabs) / 2 * 1.02, (slabs, got / build)


def test_allocation_free_ladder_rejects_sizes_beyond_its_scratch():
    """ri_ppl_noalloc checks its arguments and its fixed scratch size before any device
    call: bad arguments give RI_E_ARG / RI_E_ALIAS, sizes whose one-block-pair plan needs
    more than RI_PPL_NOALLOC_MAX_BYTES give RI_E_NOMEM with the sizes in the message."""
    from paper_1810_08142_amd import _lib
    L = _lib.lib()
    assert L.ri_ppl_noalloc(None, None, 2, 3, 4, None, 0, None) == 1
    assert L.ri_ppl_noalloc(8, 16, 2, 3, 4, 24, 7, None) == 1
    assert L.ri_ppl_noalloc(4096, 8192, 2, 3, 4, 8192, 0, None) == 2
    limit = 64 << 20
    assert f"{limit}".encode() not in L.ri_last_error_msg()
    for o, v, naux, prec in [(8, 112, 336, 0), (8, 128, 384, 0), (16, 256, 768, 2), (16, 160, 480, 2)]:
        assert L.ri_ppl_noalloc(8, 1 << 40, o, v, naux, 1 << 44, prec, None) == 3
        msg = L.ri_last_error_msg()
        assert f"o={o} v={v} naux={naux}".encode() in msg and f"{limit}".encode() in msg
