"""The HIP library loads on a machine without a GPU, exports every symbol that
include/dms.h declares, and derives the same specification constants as the
oracle (host-only calls; no kernel runs here)."""
import os
import re

import numpy as np

from oracle import oracle as O
import paper_2005_11547_amd as P
from paper_2005_11547_amd import dms

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "dms.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dms_[a-z0-9_]+)\s*\(", text)))


def test_header_matches_exports():
    names = declared_functions()
    assert len(names) >= 14
    L = P.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(dms.EXPORTS) == names


def test_library_constants_equal_oracle_constants():
    for seed in (0, 1, 2005_11547, 2 ** 64 - 1):
        for t in (1, 331, 512, 1676, 8122, 38166):
            lib = P.spec_constants(seed, t)
            keys = O.hash_keys(seed)
            assert [int(v) for v in lib["keys"]] == [keys[n] for n in
                                                     ("key_r", "key_a", "key_u", "key_v", "key_s", "key_l")]
            assert [int(v) for v in lib["pois"]] == list(O.poisson_thresholds())
            W, R, u = O.tables(t)
            assert np.array_equal(lib["W"], np.array(W)) and np.array_equal(lib["R"], np.array(R))
            assert lib["u"] == u


def test_library_tabulation_tables_equal_oracle():
    # std::mt19937_64 in the library against the oracle's own MT19937-64
    for seed in (0, 2005_11547, 2 ** 64 - 1):
        assert [int(v) for v in P.spec_tabulation(seed)] == list(O.tab_tables(seed))


def test_library_t_of_k_equals_oracle():
    for k in list(range(1, 4097)) + [8192, 65536]:
        assert P.t_of_k(k) == O.t_of_k(k), k


def test_status_strings():
    L = P.lib()
    assert L.dms_status_str(0) == b"DMS_OK"
    assert L.dms_status_str(-1) == b"DMS_EINVAL"
