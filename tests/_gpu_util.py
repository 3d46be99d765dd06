"""Helpers for the GPU parity tests: device transfer and the tolerance
checks.  The expected values always come from the FP64 oracle."""
import sys

import numpy as np
import pytest
import torch

import oracle


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def announce(*what):
    """Name the case on stdout before a GPU step (so a fault names it)."""
    print("[case]", *what, flush=True)
    sys.stdout.flush()


def dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


def dev_bf16_bits(bits):
    return torch.from_numpy(np.ascontiguousarray(bits).view(np.int16)).cuda().view(torch.bfloat16)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().to(torch.float64).numpy()


def assert_normwise(C_hat, C_ref, tol, what=""):
    err = oracle.normwise_rel_err(C_hat, C_ref)
    assert err <= tol, "%s normwise relative error %.3e > %.1e" % (what, err, tol)
    return err
