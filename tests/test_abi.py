"""C-ABI contract checks that need no GPU: the library loads, exports every function
the header declares, and rejects bad arguments before touching a device."""
import ctypes as C
import math
import os
import re

import pytest

import paper_2305_09044_amd as trd
from paper_2305_09044_amd import _lib

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = os.path.join(os.path.dirname(HERE), "include", "trd.h")


def test_header_declares_the_documented_calls():
    names = trd.header_functions(HEADER)
    for n in ["trd_create", "trd_destroy", "trd_last_error", "trd_set_problem", "trd_reconstruct",
              "trd_weights", "trd_grad", "trd_fgmc_gram", "trd_step", "trd_fit", "trd_loss_fwd",
              "trd_loss_bwd", "trd_sample_sketch", "trd_problem_info", "trd_profile",
              "trd_profile_read", "trd_set_precision", "trd_set_variant"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = trd.load()
    for n in trd.header_functions(HEADER):
        assert hasattr(lib, n), n


def test_exported_symbols_are_c_linkage():
    out = os.popen(f"nm -D --defined-only {_lib.LIB_PATH}").read()
    syms = set(re.findall(r"\bT (trd_\w+)$", out, re.M))
    assert set(trd.header_functions(HEADER)) <= syms


def test_struct_layouts_match_header(tmp_path):
    # the C compiler's view of the ABI structs must equal the ctypes mirror
    src = tmp_path / "sz.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "trd.h"\n'
        'int main(void){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(trd_sketch), sizeof(trd_fit_opts),'
        ' sizeof(trd_fit_report), offsetof(trd_fit_opts, sketch_sizes), offsetof(trd_fit_opts, seed),'
        ' offsetof(trd_sketch, idx)); return 0;}\n')
    exe = tmp_path / "sz"
    assert os.system(f"gcc -I{os.path.dirname(HEADER)} {src} -o {exe}") == 0
    got = [int(v) for v in os.popen(str(exe)).read().split()]
    want = [C.sizeof(_lib.trd_sketch), C.sizeof(_lib.trd_fit_opts), C.sizeof(_lib.trd_fit_report),
            _lib.trd_fit_opts.sketch_sizes.offset, _lib.trd_fit_opts.seed.offset,
            _lib.trd_sketch.idx.offset]
    assert got == want


def test_weights_rejects_bad_sigma_without_a_device():
    lib = trd.load()
    for s in (0.0, -1.0, float("nan")):
        assert lib.trd_weights(None, 0, 0, s, None, None) == _lib.TRD_EINVAL
    assert b"sigma" in lib.trd_last_error(None)
    assert lib.trd_weights(None, 0, 7, 1.0, None, None) == _lib.TRD_EINVAL
    assert lib.trd_weights(None, -1, 0, 1.0, None, None) == _lib.TRD_EINVAL
    # n == 0 with a valid sigma is a no-op
    assert lib.trd_weights(None, 0, 0, math.inf, None, None) == _lib.TRD_OK


def test_sample_sketch_rejects_bad_arguments():
    lib = trd.load()
    d = (C.c_int64 * 2)(10, 10)
    s = (C.c_int32 * 2)(3, 3)
    outs = (C.c_void_p * 2)(None, None)
    assert lib.trd_sample_sketch(0, 0, 0, 1, d, s, outs, None) == _lib.TRD_EINVAL   # N < 2
    assert lib.trd_sample_sketch(0, 0, 5, 2, d, s, outs, None) == _lib.TRD_EINVAL   # k out of range
    assert lib.trd_sample_sketch(0, 0, 0, 2, d, s, outs, None) == _lib.TRD_EINVAL   # NULL outputs


def test_workspace_query_checks_arguments_before_the_device():
    lib = trd.load()
    d = (C.c_int64 * 3)(10, 10, 10)
    r = (C.c_int32 * 3)(3, 3, 3)
    b = C.c_size_t()
    f32, f64 = _lib.TRD_F32, _lib.TRD_F64
    nat, bf = _lib.TRD_PREC_NATIVE, _lib.TRD_PREC_BF16
    q = lib.trd_workspace_bytes
    assert q(0, 1, d, r, f32, nat, 5, C.byref(b), None) == _lib.TRD_EUNSUPPORTED   # N < 2
    assert q(0, 3, None, r, f32, nat, 5, C.byref(b), None) == _lib.TRD_EINVAL      # NULL dims
    assert q(0, 3, d, r, f32, nat, 5, None, None) == _lib.TRD_EINVAL               # no output
    assert q(0, 3, d, r, 7, nat, 5, C.byref(b), None) == _lib.TRD_EINVAL           # dtype
    assert q(0, 3, d, r, f32, 9, 5, C.byref(b), None) == _lib.TRD_EINVAL           # precision
    assert q(0, 3, d, r, f64, bf, 5, C.byref(b), None) == _lib.TRD_EUNSUPPORTED    # BF16 on FP64
    assert q(0, 3, d, r, f32, nat, -1, C.byref(b), None) == _lib.TRD_EINVAL        # n_obs < 0
    assert q(0, 3, d, r, f32, nat, 1001, C.byref(b), None) == _lib.TRD_EINVAL      # > prod(dims)
    assert b"n_obs" in lib.trd_last_error(None)
    r[1] = 17
    assert q(0, 3, d, r, f32, nat, 5, C.byref(b), None) == _lib.TRD_EUNSUPPORTED   # rank > 16
    r[1] = 3
    import torch
    rc = q(0, 3, d, r, f32, nat, 500, C.byref(b), None)
    if torch.cuda.is_available():
        assert rc == _lib.TRD_OK and b.value > 0
    else:
        assert rc == _lib.TRD_EDEVICE   # planning needs the device's LDS and unit counts


def test_context_calls_reject_null_context():
    lib = trd.load()
    assert lib.trd_set_problem(None, 3, None, None, 0, None, None, None) == _lib.TRD_EINVAL
    assert lib.trd_step(None, None, 0, 1.0, 0.0, None, None, None, None) == _lib.TRD_EINVAL
    assert lib.trd_fit(None, None, None, None, None) == _lib.TRD_EINVAL
    assert lib.trd_profile(None, 1) == _lib.TRD_EINVAL
    assert lib.trd_set_precision(None, 0) == _lib.TRD_EINVAL
    assert lib.trd_set_variant(None, 0, 0, 0) == _lib.TRD_EINVAL
    assert lib.trd_sample_leverage(None, None, 0, 0, 0, 1, 1e-9, None, None, None) == _lib.TRD_EINVAL
    lib.trd_destroy(None)  # ignored


def test_header_constants_match_the_binding():
    txt = open(HEADER).read()
    consts = dict((m.group(1), int(m.group(2)))
                  for m in re.finditer(r"#define\s+(TRD_\w+)\s+(-?\d+)", txt))
    for name in ("TRD_OK", "TRD_EINVAL", "TRD_PREC_NATIVE", "TRD_PREC_BF16", "TRD_PREC_BF16X3",
                 "TRD_SIGMA_FIXED", "TRD_SIGMA_GIVEN", "TRD_SIGMA_QUANTILE", "TRD_DIR_SCALED",
                 "TRD_FLAG_CLAMPED", "TRD_SAMPLE_RSTS", "TRD_SAMPLE_ROWS", "TRD_SAMPLE_LEVERAGE",
                 "TRD_DIR_GRADIENT", "TRD_GRAM_GLOBAL", "TRD_GRAM_LOCAL"):
        assert getattr(_lib, name) == consts[name], name


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    bench = os.path.join(os.path.dirname(HERE), "bench.py")
    r = subprocess.run([sys.executable, bench, "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.dirname(_lib.__file__)
    for root, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(root, f)).read()
                assert "oracle" not in re.sub(r"#.*|//.*", "", txt).replace("oracle-free", ""), f


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    # no fallback: without libtrd.so every entry point raises instead of computing elsewhere
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libtrd.so"))
    with pytest.raises(ImportError, match="missing"):
        _lib.load()
    with pytest.raises(ImportError):
        _lib.trd_weights(__import__("torch").zeros(4), 1.0)
