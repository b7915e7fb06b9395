"""The fast engine hands sets to wavefronts largest first (DMS_OPT_ORDER = 1,
the default) or in input order (0).  Only the order of work changes: every
output must be identical under both, and equal to the oracle's."""
import numpy as np
import pytest

import workloads as WL
from oracle import oracle as O

pytestmark = pytest.mark.gpu

SEED = WL.HASH_SEED


@pytest.fixture(scope="module")
def torch():
    import torch
    return torch


def _ctx(order):
    from paper_2005_11547_amd import Context, dms
    c = Context(SEED)
    c.set_option(dms.OPT_ORDER, order)
    return c


def test_option_values(torch):
    from paper_2005_11547_amd import DMSError, dms
    c = _ctx(1)
    assert c.get_option(dms.OPT_ORDER) == 1.0
    c.set_option(dms.OPT_ORDER, 0)
    assert c.get_option(dms.OPT_ORDER) == 0.0
    for bad in (-1, 0.5, 2):
        with pytest.raises(DMSError):
            c.set_option(dms.OPT_ORDER, bad)
    c.close()


def test_sketch_lsh_bottomk_identical_under_both_orders(torch):
    from paper_2005_11547_amd import to_device
    # an uneven batch: Zipf sizes, a few heavy sets that are split into parts,
    # empty and invalid rows in between
    rp, idx, w = WL.uneven_k1024(seed=61, n_sets=3000)
    rows = [(idx[rp[q]:rp[q + 1]], w[rp[q]:rp[q + 1]]) for q in range(len(rp) - 1)]
    rows[10:10] = [([], []), ([3], [-1.0]), ([4, 5], [0.0, 0.0])]
    rp, idx, w = WL.csr_from_rows(rows)
    d = to_device(rp, idx, w)
    outs = []
    for order in (0, 1):
        c = _ctx(order)
        print(f"[order] {order}", flush=True)
        sk = c.sketch(*d, 256, full=True)
        lk = c.lsh(*d, 16, 4)
        bk = c.bottomk(*d, 64)
        torch.cuda.synchronize()
        outs.append({"u32": sk["u32"].cpu().numpy(), "bits": sk["bits"].cpu().numpy(),
                     "st": sk["status"].cpu().numpy(), "keys": lk["keys"].cpu().numpy(),
                     "lst": lk["status"].cpu().numpy(), "bs": bk["s"].cpu().numpy(),
                     "br": bk["rank"].cpu().numpy()})
        c.close()
    for key in outs[0]:
        assert np.array_equal(outs[0][key], outs[1][key]), key
    sample = np.arange(0, len(rp) - 1, 97)
    sub = WL.csr_from_rows([rows[q] for q in sample])
    ref = O.sketch_csr(*sub, 256, SEED)
    assert np.array_equal(outs[1]["u32"][sample].view(np.uint32), ref["u32"])
    assert np.array_equal(outs[1]["st"][sample], ref["status"])
