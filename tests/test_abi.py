"""The C-ABI library loads and exports every function include/sgpm.h declares
(no device calls)."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sgpm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(sgpm_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_core_calls():
    names = declared_functions()
    for must in ["sgpm_create", "sgpm_destroy", "sgpm_graph_from_csr", "sgpm_pattern_create", "sgpm_estimate",
                 "sgpm_estimate_batch", "sgpm_exact_count", "sgpm_gs_sparsify", "sgpm_model_train"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2405_03488_amd import sgpm as S
    L = S.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert set(S.EXPORTED) >= set(declared_functions())


def test_device_count_without_gpu_does_not_fail():
    from paper_2405_03488_amd import sgpm as S
    assert S.lib().sgpm_device_count() >= 0


def test_binding_refuses_missing_library(tmp_path, monkeypatch):
    from paper_2405_03488_amd import sgpm as S
    monkeypatch.setattr(S, "_lib", None)
    monkeypatch.setattr(S, "SO_PATH", str(tmp_path / "absent.so"))
    try:
        S.lib()
    except RuntimeError as e:
        assert "missing" in str(e)
    else:
        raise AssertionError("binding loaded a missing library")
