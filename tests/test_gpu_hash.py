"""The GPU's hash family against the Python-integer one (Sec. 3.1 H1;
Sec. 3.2 DH0 and eq. (2)), with no oracle in between: a window of the pin
keys is sketched on the GPU by both update kernels and compared word for word
with the sketch built from the Python-integer hashes."""
import numpy as np
import pytest
import torch

from paper_1803_11449_amd import ddhf, traffic
from test_hash_pins import SETS, pin_keys, python_sketch

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.mark.parametrize("path", [1, 2], ids=["direct", "binned"])
@pytest.mark.parametrize("shape", SETS)
def test_gpu_sketch_equals_python_hashes(shape, path):
    g, k, r, alpha = shape
    print(f"hash pin on GPU: shape={shape} path={path}", flush=True)
    keys = pin_keys()
    # every key as a source once and as a destination once
    dsts = np.roll(keys, 17)
    pairs = np.stack([keys, dsts], axis=1).astype(np.uint32)
    want = python_sketch(g, k, r, alpha, traffic.HASH_SEED, pairs)
    with ddhf.Sketch(g, k, r, alpha, traffic.HASH_SEED, device=0) as sk:
        sk.set_option(ddhf.SKETCH_OPT_UPDATE_PATH, path)
        sk.update(torch.from_numpy(pairs.view(np.int32)).to(DEV))
        torch.cuda.synchronize()
        got = sk.download()
    diff = np.nonzero(got != want)[0]
    assert diff.size == 0, (int(diff[0]), int(got[diff[0]]), int(want[diff[0]]))
