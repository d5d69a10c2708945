"""GPU parity on the input types and reorderings of the paper's comparison tests
(SVI): every type under every reordering, keys bit-identical to the oracle's."""
import numpy as np
import pytest

import tsqs_inputs as ti
from gpu_util import gpu_sort, gpu_sort_pairs, payload_valid, same_bits

pytestmark = pytest.mark.gpu

N = (1 << 20) + 37


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_00558_amd as tsqs
    tsqs.load_library()
    yield


@pytest.mark.parametrize("order", ti.PAPER_ORDERS)
@pytest.mark.parametrize("kind", ti.PAPER_TYPES)
def test_paper_inputs_int32(oracle_mod, kind, order):
    print("case: paper input", kind, order, N, flush=True)
    k = ti.paper_input(kind, order, N, 1 << 16, dtype="int32", seed=21)
    assert same_bits(gpu_sort(k), oracle_mod.sort(k))


@pytest.mark.parametrize("m", [2, 64, 1 << 30])
@pytest.mark.parametrize("kind", ["random", "sawtooth", "plateau", "hill"])
def test_paper_inputs_value_ranges(oracle_mod, kind, m):
    """Few distinct values (long equal bands) to almost all distinct, with payloads."""
    print("case: paper input range", kind, m, flush=True)
    for order in ("as_is", "fort", "dither"):
        k = ti.paper_input(kind, order, N, m, dtype="int64", seed=22)
        v = np.arange(N, dtype=np.uint32)
        gk, gv = gpu_sort_pairs(k, v)
        assert same_bits(gk, oracle_mod.sort(k)), order
        assert payload_valid(k, gk, gv), order


@pytest.mark.parametrize("order", ["fort", "front_half_reversed", "back_half_reversed"])
def test_paper_inputs_float32(oracle_mod, order):
    print("case: paper input float32", order, flush=True)
    k = ti.paper_input("organ_pipes", order, N, 1 << 20, dtype="float32", seed=23)
    assert same_bits(gpu_sort(k), oracle_mod.sort(k))
