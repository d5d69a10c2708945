"""Helpers of the GPU tests: numpy <-> device tensors, comparison against the oracle."""
import numpy as np

CODES = {np.dtype(np.int32): 0, np.dtype(np.uint32): 1, np.dtype(np.int64): 2,
         np.dtype(np.uint64): 3, np.dtype(np.float32): 4}
SIGNED = {4: np.int32, 8: np.int64}


def to_dev(a):
    import torch
    a = np.ascontiguousarray(a)
    view = a.view(SIGNED[a.dtype.itemsize]) if a.dtype != np.float32 else a
    return torch.from_numpy(view.copy()).to("cuda:0")


def from_dev(t, dtype):
    return t.cpu().numpy().view(np.dtype(dtype))


def device_ok():
    """The last call reported no device error (its statistics wait for it)."""
    import paper_1505_00558_amd as tsqs
    rc, st = tsqs.last_call_status()
    assert rc == tsqs.OK and st["error_flags"] == 0, (rc, st["error_flags"])
    return st


def gpu_sort(a):
    import paper_1505_00558_amd as tsqs
    import torch
    t = to_dev(a)
    tsqs.sort(t, CODES[np.dtype(a.dtype)])
    torch.cuda.synchronize()
    if a.size > 1:
        device_ok()
    return from_dev(t, a.dtype)


def gpu_sort_pairs(a, v):
    import paper_1505_00558_amd as tsqs
    import torch
    t = to_dev(a)
    tv = to_dev(np.asarray(v, dtype=np.uint32))
    tsqs.sort_pairs(t, tv, CODES[np.dtype(a.dtype)])
    torch.cuda.synchronize()
    if a.size > 1:
        device_ok()
    return from_dev(t, a.dtype), from_dev(tv, np.uint32)


def bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint8).reshape(a.size, -1) if a.size else a.view(np.uint8).reshape(0, 1)


def same_bits(x, y):
    return x.shape == y.shape and np.array_equal(bits(x), bits(y))


def payload_valid(keys_in, keys_out, vals_out):
    """vals_out is a permutation of 0..n-1 and keys_in[vals_out[i]] == keys_out[i]."""
    n = keys_in.size
    if not np.array_equal(np.sort(vals_out), np.arange(n, dtype=np.uint32)):
        return False
    return np.array_equal(bits(keys_in)[vals_out.astype(np.int64)], bits(keys_out))
