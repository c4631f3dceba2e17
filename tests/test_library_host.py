"""Host-side checks of libhrir.so that need no GPU: every symbol the header
declares is exported, the FP64 factorization agrees with the oracle from the
same G0, and argument errors come back as status codes."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_1502_03162_amd as H
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", fn)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M):
            if m.group(1) not in ("if", "defined"):
                names.append(m.group(1))
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    names = header_functions()
    assert "spconv_render" in names and "hrir_factorize" in names
    lib = ctypes.CDLL(H.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_factorize_matches_oracle_same_g0():
    hs = synth.hrir_set(2, 2, 5)
    X = hs.h
    n, m = X.shape
    lf, k, T = 32, 16, 60
    G0 = oracle.rand_g0(9, n, m - lf + 1)
    lib = H.factorize(X, lf, T, k, g0=G0, lambda0=0.2)
    f, G, tr = oracle.factorize(X, lf, T, G0, 0.2)
    assert np.max(np.abs(lib["f"] - f)) < 1e-10
    assert np.max(np.abs(lib["G"] - G)) < 1e-10 * np.max(G)
    assert np.max(np.abs(lib["cost"] - tr) / tr) < 1e-10
    rec_lib = oracle.reconstruct(lib["f"], lib["G"])
    rec_or = oracle.reconstruct(f, G)
    assert np.linalg.norm(rec_lib - rec_or) / np.linalg.norm(rec_or) < 1e-8
    p, g, nnz = oracle.topk(G, k)
    assert np.array_equal(lib["p"], p) and np.array_equal(lib["nnz"], nnz)
    gr = oracle.refit(X, f, p, nnz)
    assert np.max(np.abs(lib["g"] - gr.astype(np.float32))) <= 2e-7 * np.max(gr)
    # reported error of the kept taps
    rec = oracle.reconstruct(f, oracle.scatter_taps(p, gr, m - lf + 1))
    e = np.array([oracle.e_db(X[i], rec[i]) for i in range(n)])
    assert np.max(np.abs(lib["err_db"] - e)) < 1e-6


def test_factorize_raw_gains_without_refit():
    hs = synth.hrir_set(4, 2, 2)
    G0 = oracle.rand_g0(1, 8, 169)
    lib = H.factorize(hs.h, 32, 20, 8, g0=G0, refit=False)
    p, g, nnz = oracle.topk(lib["G"], 8)
    assert np.array_equal(lib["p"], p)
    assert np.array_equal(lib["g"], g.astype(np.float32))


def test_factorize_seed_equals_splitmix_g0():
    hs = synth.hrir_set(5, 1, 3)
    a = H.factorize(hs.h, 32, 5, 4, seed=123)
    b = H.factorize(hs.h, 32, 5, 4, g0=oracle.rand_g0(123, 6, 169))
    assert np.array_equal(a["G"], b["G"]) and np.array_equal(a["f"], b["f"])


def test_factorize_errors():
    X = np.ones((4, 20))
    with pytest.raises(H.HrirError) as e:
        H.factorize(X, 25, 3, 2)                     # lf > m
    assert e.value.code == H.HRIR_EINVAL
    with pytest.raises(H.HrirError) as e:
        H.factorize(X, 5, 3, 17)                     # k > lg = 16
    assert e.value.code == H.HRIR_EINVAL
    with pytest.raises(H.HrirError) as e:
        H.factorize(X, 5, 3, 2, g0=np.zeros((4, 16)))  # G0 must be > 0
    assert e.value.code == H.HRIR_EINVAL
    with pytest.raises(H.HrirError) as e:
        H.factorize(np.zeros((4, 20)), 5, 3, 2)      # f vanishes
    assert e.value.code == H.HRIR_ENOTPD
    Xn = X.copy(); Xn[1, 3] = np.nan
    with pytest.raises(H.HrirError) as e:
        H.factorize(Xn, 5, 3, 2)
    assert e.value.code == H.HRIR_EINVAL
    assert "not finite" in str(e.value)


def test_plan_argument_errors_before_any_device_call():
    r = np.ones(4, dtype=np.float32)
    ok_p = np.zeros((2, 3), dtype=np.int32)
    ok_g = np.ones((2, 3), dtype=np.float32)
    for args, msg in [
        ((r, np.full((2, 3), 9, dtype=np.int32), ok_g, 9), "outside"),       # p >= lg
        ((r, -ok_p - 1, ok_g, 9), "outside"),                                 # p < 0
        ((r, ok_p, -ok_g, 9), ">= 0"),                                        # negative gain
        ((np.ones(65, dtype=np.float32), ok_p, ok_g, 9), "lf=65"),           # lf too long
        ((r, np.zeros((2, 65), dtype=np.int32), np.zeros((2, 65), dtype=np.float32), 9), "k=65"),
        ((r, ok_p, ok_g, 0), "lg=0"),
    ]:
        with pytest.raises(H.HrirError) as e:
            H.Plan(*args)
        assert e.value.code == H.HRIR_EINVAL and msg in str(e.value)


def test_stream_calls_reject_null_handles():
    lib = H.lib()
    hd = ctypes.c_void_p()
    assert lib.stream_open(None, 4, 1 << 24, 0, ctypes.byref(hd)) == H.HRIR_EINVAL
    assert lib.stream_submit(None, 0, None, 1, 0, 1, 0) == H.HRIR_EINVAL
    assert lib.stream_end(None, 0, 0, 1, 0) == H.HRIR_EINVAL
    assert lib.stream_poll(None, None, 0, 0) == H.HRIR_EINVAL
    assert lib.stream_info(None, None) == H.HRIR_EINVAL
    assert lib.stream_loadgen(None, None, None) == H.HRIR_EINVAL
    lib.stream_close(None)                              # no-op


def test_struct_layouts_match_the_header(tmp_path):
    """sizeof/offsetof of every struct of the ABI, from a C program compiled
    against the header, equal the binding's ctypes layouts."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"spconv_job": H.SpconvJob, "block_job": H.BlockJob, "hrir_result": H.HrirResult,
               "stream_load": H.StreamLoad, "stream_load_stats": H.StreamLoadStats}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "hrir.h"', "int main(void) {"]
    for name, ct in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in ct._fields_:
            lines.append(f'printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        a, b, c = line.split()
        got[(a, b)] = int(c)
    for name, ct in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(ct), name
        for field, _ in ct._fields_:
            assert got[(name, field)] == getattr(ct, field).offset, (name, field)


def test_surrogate_select_brute_force():
    """The fallback rule against a brute-force evaluation of its definition."""
    rng = np.random.default_rng(9)
    q_az, q_el = rng.uniform(-1.4, 1.4, 500), rng.uniform(-0.8, 4.0, 500)
    v_az, v_el = rng.uniform(-1.4, 1.4, 60), rng.uniform(-0.8, 4.0, 60)
    m_az, m_el = rng.uniform(-1.4, 1.4, 90), rng.uniform(-0.8, 4.0, 90)
    err = rng.uniform(-45, -15, 60)
    ch = H.surrogate_select(q_az, q_el, v_az, v_el, err, m_az, m_el, -30.0)

    def unit(a, e):
        return np.stack([np.sin(a), np.cos(a) * np.cos(e), np.cos(a) * np.sin(e)], axis=-1)

    Q, V, Mm = unit(q_az, q_el), unit(v_az, v_el), unit(m_az, m_el)
    for i in range(500):
        nv = int(np.argmax(V @ Q[i]))
        want = int(np.argmax(Mm @ Q[i])) if err[nv] > -30.0 else -1
        assert ch[i] == want
    assert 0 < np.sum(ch >= 0) < 500
    with pytest.raises(H.HrirError):
        H.surrogate_select(q_az, q_el, [], [], [], m_az, m_el)


def test_region_labels_are_validated_before_any_device_call():
    r = np.ones((2, 4), dtype=np.float32)
    p = np.zeros((3, 2), dtype=np.int32)
    g = np.ones((3, 2), dtype=np.float32)
    for regions in ([0, 2, 1], [0, -1, 1]):
        with pytest.raises(H.HrirError) as e:
            H.Plan(r, p, g, 9, regions=regions)
        assert e.value.code == H.HRIR_EINVAL and "region" in str(e.value)
    with pytest.raises(H.HrirError):
        H.Plan(r, p, g, 9)                                  # two resonance filters need labels


def test_product_code_never_uses_the_oracle():
    """The oracle is test infrastructure: no source of the package (Python or
    native) imports, loads or calls it."""
    import pathlib
    pkg = pathlib.Path(__file__).resolve().parents[1] / "paper_1502_03162_amd"
    offenders = []
    for f in pkg.rglob("*"):
        if f.suffix not in (".py", ".hip", ".cpp", ".h") or "_build" in f.parts:
            continue
        text = f.read_text()
        if "import oracle" in text or "from oracle" in text or "liboracle" in text or "or_sparse" in text:
            offenders.append(str(f))
    assert not offenders, offenders


def test_bench_refuses_several_gpus():
    import json
    import pathlib
    import subprocess
    import sys
    root = pathlib.Path(__file__).resolve().parents[1]
    res = subprocess.run([sys.executable, str(root / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                         timeout=120)
    assert res.returncode != 0
    assert "one GPU" in json.loads(res.stdout.strip().splitlines()[-1])["error"]
