"""CPU-side checks of the C ABI: the library loads, exports every function
that include/kvs.h declares, and reports a device error (not a crash) when
no GPU is present."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "kvs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kvs_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("kvs_create", "kvs_set_material", "kvs_set_force", "kvs_project", "kvs_step", "kvs_read_traces"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2607_28414_amd import kvs
    L = kvs.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    # and the binding wraps every one of them with the same name
    assert set(declared_functions()) <= set(kvs.SIGNATURES)


def test_status_strings():
    from paper_2607_28414_amd import kvs
    L = kvs.lib()
    assert L.kvs_status_string(0) == b"ok"
    assert L.kvs_status_string(6).startswith(b"time step")


def test_create_without_gpu_is_a_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2607_28414_amd import kvs
    with pytest.raises(kvs.KvsError) as e:
        kvs.kvs_create((8, 8, 8, 1e-3, 1e-3, 1e-3))
    assert e.value.status == kvs.KVS_EDEVICE


def test_create_rejects_bad_grid_before_touching_the_device():
    from paper_2607_28414_amd import kvs
    with pytest.raises(kvs.KvsError) as e:
        kvs.kvs_create((2, 8, 8, 1e-3, 1e-3, 1e-3))
    assert e.value.status == kvs.KVS_EINVAL
    with pytest.raises(kvs.KvsError) as e:
        kvs.kvs_create((8, 8, 8, 1e-3, 0.0, 1e-3))
    assert e.value.status == kvs.KVS_EINVAL
