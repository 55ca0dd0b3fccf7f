"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every function include/ccgpu.h declares, its sampler matches the oracle's
independent implementation of the same published generator, and argument
errors come back as status codes."""
import os
import re

import numpy as np
import pytest

import oracle
import paper_1409_0035_amd as cc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "ccgpu.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cc_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    lib = cc.load_library()
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(cc.EXPORTED)


@pytest.mark.parametrize("n,k,seed", [(10, 10, 0), (10_000, 64, 1), (1 << 20, 256, 2), (4_194_304, 128, 4),
                                      (97, 1, 123456789), (2 ** 31 - 1, 300, 2 ** 63 + 5)])
def test_sampler_matches_oracle(n, k, seed):
    a = cc.cc_draw_samples(n, k, seed)
    b = np.array(oracle.draw_samples(n, k, seed), dtype=np.int32)
    assert (a == b).all()


@pytest.mark.parametrize("case", range(12))
def test_weighted_sampler_matches_oracle(case):
    """The library's node-weighted sample (host code) equals the oracle's
    independent implementation: same ids, light flags and tau."""
    rng = np.random.default_rng(500 + case)
    n = int(rng.integers(1, [40, 400, 5000][case % 3]))
    hi = [2, 10, 1000, 2 ** 20][case % 4]
    beta = rng.integers(0, hi, size=n).astype(np.uint32)
    if case % 5 == 0:
        beta[int(rng.integers(0, n))] = 3_000_000
    if not beta.any():
        beta[0] = 1
    k = int(rng.integers(1, max(2, min(n, 300))))
    a = cc.cc_draw_weighted(beta, k, 900 + case)
    b = oracle.draw_weighted([int(x) for x in beta], k, 900 + case)
    assert list(a[0]) == list(b[0]) and list(a[1]) == list(b[1]) and a[2:] == b[2:]


def test_weighted_sampler_rejects_bad_arguments():
    with pytest.raises(cc.CCError) as e:
        cc.cc_draw_weighted(np.zeros(10, np.uint32), 3, 1)
    assert e.value.status == cc.CC_EINVAL
    with pytest.raises(cc.CCError):
        cc.cc_draw_weighted(np.ones(10, np.uint32), 0, 1)


def test_sampler_rejects_bad_arguments():
    with pytest.raises(cc.CCError) as e:
        cc.cc_draw_samples(5, 6, 1)
    assert e.value.status == cc.CC_EINVAL
    with pytest.raises(cc.CCError):
        cc.cc_draw_samples(5, 0, 1)


def test_status_strings():
    for s in range(9):
        assert cc.cc_status_str(s) != "unknown status"


def test_context_without_device_is_an_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(cc.CCError) as e:
        cc.cc_context_create(0)
    assert e.value.status == cc.CC_EDEVICE


def test_tuning_calls_reject_null_arguments():
    """Argument checks that happen before any device work."""
    lib = cc.load_library()
    t = cc.cc_tuning()
    assert lib.cc_graph_get_tuning(None, None) == cc.CC_EINVAL
    assert lib.cc_graph_set_tuning(None, None) == cc.CC_EINVAL
    assert lib.cc_autotune(None, None, 4, 0, 1, None, None) == cc.CC_EINVAL
    assert lib.cc_graph_get_tuning(None, t) == cc.CC_EINVAL
    assert cc.TUNING_FIELDS == ("alpha", "level_blocks", "scatter_blocks", "delta", "round_blocks", "local_passes")
