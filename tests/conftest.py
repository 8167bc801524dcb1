import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def pytest_report_header(config):
    return f"repo root: {ROOT}"


# ------------------------------------------------------------------ training pairs
N_TRAIN, N_HELD = 10_000, 128
HELD0 = 100_000


def make_pairs(first, count):
    """Synthetic degrade -> restore pairs from the oracle (inputs, targets) as float32 arrays."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    from oracle import pairs as op
    with ThreadPoolExecutor(16) as ex:
        res = list(ex.map(op.make_pair, range(first, first + count)))
    return np.stack([r[0] for r in res]), np.stack([r[1] for r in res])


@pytest.fixture(scope="session")
def pair_data():
    """Training pairs 0..N_TRAIN-1 (10k, drawn over 16 worker processes) and held-out pairs
    from HELD0, on the GPU (shared by the training tests of both generators)."""
    import time

    import torch
    from oracle import pairs as op
    print("generating training pairs", flush=True)
    t = time.time()
    xtr, ttr = op.make_pairs_parallel(0, N_TRAIN, workers=16)
    xte, tte = make_pairs(HELD0, N_HELD)
    print(f"pairs ready in {time.time() - t:.1f}s", flush=True)
    cuda = lambda a: torch.from_numpy(a).cuda()
    return cuda(xtr), cuda(ttr), cuda(xte), cuda(tte)
