"""Seeded code construction, encoders and the AWGN workload."""
import numpy as np
import pytest

from paper_2305_05286_amd.workload import (CHUNK, CODE_NAMES, encode, get_code, gf2_rank,
                                           has_4cycle, make_frames, sigma2_for)
from paper_2305_05286_amd.workload.registry import _build

from helpers import syndrome


@pytest.mark.parametrize("name", CODE_NAMES)
def test_encoder_produces_codewords(name):
    code = get_code(name)
    rng = np.random.default_rng(0)
    info = rng.integers(0, 2, size=(8, code.K), dtype=np.uint8)
    cw = encode(code, info)
    assert cw.shape == (8, code.N)
    assert (syndrome(code, cw) == 0).all()
    assert np.array_equal(cw[:, code.info_pos], info)


@pytest.mark.parametrize("name", [n for n in CODE_NAMES if n != "qc26112"])
def test_no_4cycles(name):
    code = get_code(name)
    assert not has_4cycle(code.row_ptr, code.col_idx)


def test_qc26112_base_has_no_4cycles():
    code = get_code("qc26112")
    sh = code.shifts
    mb, nb = sh.shape
    for r1 in range(mb):
        for r2 in range(r1 + 1, mb):
            both = np.nonzero((sh[r1] >= 0) & (sh[r2] >= 0))[0]
            for i in range(len(both)):
                for j in range(i + 1, len(both)):
                    b1, b2 = both[i], both[j]
                    assert (sh[r1, b1] - sh[r1, b2] + sh[r2, b2] - sh[r2, b1]) % code.Z != 0


def test_workload_shapes():
    c1 = get_code("reg36_n96")
    assert (c1.N, c1.M, c1.K, c1.E) == (96, 48, 48, 288)
    assert set(c1.row_degrees()) == {6} and set(c1.col_degrees()) == {3}
    assert gf2_rank(c1.dense()) == 48
    c2 = get_code("qc2304")
    assert (c2.N, c2.M, c2.K, c2.Z) == (2304, 1152, 1152, 96)
    assert c2.shifts.shape == (12, 24)
    assert set(np.unique(c2.col_degrees())) <= {2, 3, 4, 5, 6}
    assert gf2_rank(c2.dense()) == 1152
    c3 = get_code("qc26112")
    assert (c3.N, c3.M, c3.K, c3.Z) == (26112, 17664, 8448, 384)
    assert c3.shifts.shape == (46, 68)
    assert c3.col_degrees().min() == 1  # the last staircase column


def test_frozen_artefacts_reproduce_from_seed():
    for name in ["reg36_n96", "qc2304", "qc_t16"]:
        a = get_code(name)
        b = _build(name)
        assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col_idx, b.col_idx)


def test_frames_prefix_and_statistics():
    code = get_code("qc_t16")
    l1, c1 = make_frames(code, 1.5, 100, key=(3, 1))
    l2, c2 = make_frames(code, 1.5, CHUNK + 50, key=(3, 1))
    assert np.array_equal(l1, l2[:100]) and np.array_equal(c1, c2[:100])
    l3, _ = make_frames(code, 1.5, 50, key=(3, 1), start=CHUNK)
    assert np.array_equal(l3, l2[CHUNK:])
    s2 = sigma2_for(code, 1.5)
    z = l2.astype(np.float64) * (1 - 2.0 * c2)  # = 2/s2 + (2/s2) sigma n
    assert abs(z.mean() / (2 / s2) - 1) < 0.01
    assert abs(z.var() / (4 / s2) - 1) < 0.02
    assert l2.dtype == np.float32


# ---- mixed-code workload ---------------------------------------------------

def test_mixed_family_shapes_and_codewords():
    from paper_2305_05286_amd.workload import RATES, Z_VALUES, make_mixed_batch, mixed_family
    fam = mixed_family()
    assert len(fam) == len(RATES) * len(Z_VALUES)
    rates = sorted({round(c.K / c.N, 4) for c in fam})
    assert rates == sorted(round(k, 4) for k in (1 / 3, 1 / 2, 2 / 3, 5 / 6, 8 / 9))
    assert sorted({c.Z for c in fam}) == list(Z_VALUES)
    for c in fam:
        assert c.M == c.N - c.K                       # staircase parity part: full rank
        mb, nb = c.shifts.shape
        kb = nb - mb
        par = (c.shifts[:, kb:] >= 0).astype(int)     # strict lower dual-diagonal
        assert (par == np.eye(mb, dtype=int) + np.eye(mb, k=-1, dtype=int)).all()
    b = make_mixed_batch(fam, 600, key=(9,))
    assert b["llr"].dtype == np.float32 and b["offset"].dtype == np.int64
    lens = np.array([fam[i].N for i in b["code"]])
    assert (np.diff(b["offset"]) == lens[:-1]).all() and b["offset"][0] == 0
    assert b["llr"].size == lens.sum()
    assert (b["ebn0"] >= 0).all() and (b["ebn0"] <= 4).all()
    assert len(set(b["code"].tolist())) == len(fam)    # 600 frames reach every code
    for c in range(len(fam)):
        fr = np.nonzero(b["code"] == c)[0][:3]
        words = np.stack([b["codeword"][b["offset"][f]:b["offset"][f] + fam[c].N] for f in fr])
        assert (syndrome(fam[c], words) == 0).all()
        # LLR sign follows the codeword at high SNR on average
        llr = np.concatenate([b["llr"][b["offset"][f]:b["offset"][f] + fam[c].N] for f in fr])
        assert ((llr < 0) == np.concatenate(list(words)).astype(bool)).mean() > 0.8
    again = make_mixed_batch(fam, 600, key=(9,))
    assert (again["llr"] == b["llr"]).all() and (again["code"] == b["code"]).all()
