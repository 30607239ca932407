"""Host-side checks of libgmf: it loads, exports every declared symbol, and its
host logic (configuration, workspace planning, seeded schedule) is right.
No kernel is launched here."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2412_20509_amd", "libgmf.so")


def _declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"\b(gmf_[a-z0-9_]+)\s*\(", txt):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libgmf.so is not built (run __graft_entry__.build())")
    from paper_2412_20509_amd import gmf
    return gmf


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "libgmf.so is not built"
    so = ctypes.CDLL(LIB)
    names = _declared_symbols()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(so, n)]
    assert not missing, missing


def test_config_defaults(lib):
    c = lib.gmf_config_default()
    assert (c.family, c.link, c.precision, c.bias_mode) == (0, 0, 0, 0)
    assert (c.R, c.S, c.d) == (10, 5, 1)
    assert list(c.lambda_) == [0.0, 0.0, 1.0, 1.0]
    assert (c.rate0, c.decay, c.tau) == (0.05, 0.05, 0.75)
    assert (c.alpha1, c.alpha2, c.damping, c.eps) == (0.1, 0.01, 1e-3, 1e-8)


def _cfg(lib, **kw):
    c = lib.gmf_config_default()
    c.n, c.m, c.d, c.p, c.q = 1000, 500, 5, 1, 1
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def test_workspace_bytes_scale_and_reject_bad_configs(lib):
    base = lib.gmf_workspace_bytes(_cfg(lib))
    assert base > 1000 * 500 * 4
    assert lib.gmf_workspace_bytes(_cfg(lib), True) >= base + 1000 * 500 * 4
    big = lib.gmf_workspace_bytes(_cfg(lib, n=10_000, m=2_000, d=10, p=3))
    assert big > 10_000 * 2_000 * 4
    for bad in (dict(d=0), dict(p=40, q=20, d=10), dict(R=0), dict(S=600),
                dict(family=2, link=0), dict(family=1, link=1), dict(alpha1=0.0),
                dict(phi=-1.0), dict(precision=7), dict(bias_mode=1, alpha1=1.0)):
        assert lib.gmf_workspace_bytes(_cfg(lib, **bad)) == 0, bad


def test_schedule_matches_oracle_generator(lib):
    from oracle import gmf_oracle as G
    for seed, n, m, R in [(2001, 1000, 500, 10), (7, 37, 23, 4), (2**63 + 5, 5, 3, 2)]:
        rp, cp, rr = lib.gmf_schedule_host(seed, n, m, R, 1, 300)
        assert np.array_equal(rp, G.permutation(seed, G.STREAM_ROWS, n))
        assert np.array_equal(cp, G.permutation(seed, G.STREAM_COLS, m))
        want = [G.row_block_draw(seed, t, R) for t in range(1, 301)]
        assert rr.tolist() == want
    # a later window of the draws
    _, _, rr = lib.gmf_schedule_host(99, 10, 10, 10, 12345, 7)
    assert rr.tolist() == [G.row_block_draw(99, t, 10) for t in range(12345, 12352)]


def test_product_path_does_not_touch_oracle():
    """The package and its native sources never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_2412_20509_amd")
    for path in glob.glob(os.path.join(pkg, "**", "*.*"), recursive=True):
        if path.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
            txt = open(path).read()
            assert "oracle" not in txt.lower(), path


def test_tune_table_round_trip_and_lookup(lib, tmp_path):
    """The tile-rows table (host logic only): load, lookup by shape class, the
    workspace size follows the tuned rows, save/load round trip, bad lines."""
    from paper_2412_20509_amd import gmf as M
    cfg = M.gmf_config_default()
    cfg.family, cfg.n, cfg.m, cfg.d, cfg.p, cfg.q = M.GMF_NEGBIN, 10000, 2000, 10, 3, 1
    M.tune_table_clear()
    assert M.tune_lookup(cfg) == 0
    auto_bytes = M.gmf_workspace_bytes(cfg)
    # class of this cfg: FP32, NB, stride 16, ceil(log2 1000) = 10, ceil(log2 400) = 9
    path = tmp_path / "tune.txt"
    path.write_text("# comment\n0 1 16 10 9 128 3.5\n0 1 16 11 9 64 9.0\n")
    M.tune_table_load(path)
    assert M.tune_lookup(cfg) == 128
    cfg2 = M.gmf_config_default()
    cfg2.family, cfg2.n, cfg2.m, cfg2.d, cfg2.p, cfg2.q = M.GMF_NEGBIN, 20000, 2000, 10, 3, 1
    assert M.tune_lookup(cfg2) == 64
    tuned_bytes = M.gmf_workspace_bytes(cfg)
    cfg.tile_rows = 128
    assert tuned_bytes == M.gmf_workspace_bytes(cfg)       # same plan as an explicit 128
    cfg.tile_rows = 0
    assert tuned_bytes != auto_bytes
    out = tmp_path / "saved.txt"
    M.tune_table_save(out)
    M.tune_table_clear()
    assert M.tune_lookup(cfg) == 0
    M.tune_table_load(out)
    assert M.tune_lookup(cfg) == 128 and M.tune_lookup(cfg2) == 64
    bad = tmp_path / "bad.txt"
    bad.write_text("0 1 16 10 9 100 1.0\n")                 # not a multiple of 32
    with pytest.raises(M.GMFError):
        M.tune_table_load(bad)
    assert M.tune_lookup(cfg) == 128                          # unchanged by the failed load
    M.tune_table_clear()


@pytest.mark.parametrize("struct", ["gmf_config", "gmf_mlp_config"])
def test_header_compiles_and_struct_layout_matches_binding(tmp_path, struct):
    """include/gmf.h compiles as C and as C++, and the binding's structures
    have the C structs' sizes and field offsets (the ABI the ctypes calls rely
    on)."""
    import shutil
    import subprocess
    from paper_2412_20509_amd import gmf as M
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("gcc not found")
    cls = getattr(M, struct)
    fields = [f[0] for f in cls._fields_]
    c_names = {"lambda_": "lambda"}
    src = tmp_path / "layout.c"
    body = "\n".join(f'  printf("{f} %zu\\n", offsetof({struct}, {c_names.get(f, f)}));' for f in fields)
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "gmf.h"\n'
                   f'int main(void) {{\n  printf("size %zu\\n", sizeof({struct}));\n' + body +
                   '\n  return 0;\n}\n')
    exe = tmp_path / "layout"
    inc = os.path.join(ROOT, "include")
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", inc, str(src), "-o", str(exe)], check=True)
    subprocess.run(["g++", "-fsyntax-only", "-x", "c++", "-I", inc, str(src)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                       text=True).stdout.splitlines())
    assert int(out["size"]) == ctypes.sizeof(cls)
    for f in fields:
        assert int(out[f]) == getattr(cls, f).offset, f


def _header_prototypes():
    """name -> number of parameters of every gmf_* function declared in include/*.h."""
    protos = {}
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        for m in re.finditer(r"\b(gmf_[a-z0-9_]+)\s*\(([^;{]*?)\)\s*;", txt):
            args = m.group(2).strip()
            protos[m.group(1)] = 0 if args in ("", "void") else args.count(",") + 1
    return protos


def test_binding_signatures_match_header(lib):
    """Every function the Python binding declares is in the header, with the
    same number of parameters, and every header function is bound."""
    protos = _header_prototypes()
    assert len(protos) >= 40
    so = lib.load_library()
    for n, nargs in protos.items():
        fn = getattr(so, n)
        assert fn.argtypes is not None, f"{n} is not bound"
        assert len(fn.argtypes) == nargs, (n, len(fn.argtypes), nargs)


@pytest.mark.parametrize("name,extra", [
    ("gmf_step", (1,)), ("gmf_set_precision", (0,)), ("gmf_fit", (1, 0.0, 1, None, None)),
    ("gmf_run", (1, 1, None, None)), ("gmf_deviance", (None, None)),
    ("gmf_row_deviance", (None,)), ("gmf_block_deviance", (None, 1)),
    ("gmf_get_params", (None, None, None, None, 0)), ("gmf_set_params", (None, None, None, None)),
    ("gmf_get_moments", (None, None, None, None)), ("gmf_get_schedule", (None, None, 1, 1, None)),
    ("gmf_project", (None, 0, None, 0, 1, None, None, None, 1, 0, None, None, None)),
    ("gmf_project_warm", (None, 0, None, 0, 1, None, None, 1, 1, None, None, None, None, None)),
    ("gmf_batch_run", (1, 1, None)), ("gmf_set_trace", (None, 0)), ("gmf_set_timing", (1,)),
    ("gmf_get_timing", (None, None, None)), ("gmf_sync", ()),
    ("gmf_get_timing_by_kind", (None, None)), ("gmf_compact_counts", ()),
])
def test_null_handle_is_rejected_without_touching_the_device(lib, name, extra):
    """A NULL context (or batch) handle is an argument error (GMF_EINVAL, with a
    message), checked before any device work, so this runs without a GPU."""
    so = lib.load_library()
    rc = getattr(so, name)(None, *extra)
    assert rc == lib.GMF_EINVAL, (name, rc)
    assert b"NULL" in so.gmf_last_error(), name


def test_null_handles_elsewhere(lib):
    so = lib.load_library()
    assert so.gmf_steps_done(None) == -1
    assert so.gmf_project_workspace_bytes(None, 100) == 0
    so.gmf_destroy(None)
    so.gmf_batch_destroy(None)
    so.gmf_encoder_destroy(None)
    for name, extra in (("gmf_encoder_train", (None, 0, None, 1, 1, None)),
                        ("gmf_encoder_forward", (None, 0, 1, None, 1)),
                        ("gmf_encoder_loss_grad", (None, 0, None, 1, None, None)),
                        ("gmf_encoder_get_weights", (None,) * 6)):
        assert getattr(so, name)(None, *extra) == lib.GMF_EINVAL, name
        assert so.gmf_encoder_last_error(), name


def test_rank_eigengap_matches_oracle(lib):
    """gmf_rank_eigengap (pure host code) against the oracle's estimator on
    spectra with 0 to 7 planted factors, and its argument checks."""
    from oracle import rank_oracle as K
    for d, seed in [(0, 1), (2, 2), (4, 3), (7, 4)]:
        rng = np.random.default_rng(seed)
        E = rng.normal(size=(400, 200))
        if d:
            P = np.linalg.qr(rng.normal(size=(400, d)))[0]
            Q = np.linalg.qr(rng.normal(size=(200, d)))[0]
            E += (P * (0.35 * np.sqrt(400 * 200) * np.linspace(1.0, 0.6, d))) @ Q.T
        lam = np.linalg.svd(E, compute_uv=False) ** 2
        for rmax in (8, 12):
            assert lib.rank_eigengap(lam, rmax) == K.eigengap_rank(lam, rmax)
    with pytest.raises(lib.GMFError):
        lib.rank_eigengap(np.arange(10.0), 3)          # ascending
    with pytest.raises(lib.GMFError):
        lib.rank_eigengap(np.arange(10.0)[::-1], 8)    # fewer than rmax + 5 values
    assert lib.rank_select_cv([[0.5, 0.7], [0.4, 0.6], [0.45, 0.7]]) == 1
