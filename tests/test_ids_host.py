"""The IDs path's host mapping step (dnatok_ids_map: host memory only, no
GPU) against the oracle: the table encode of every row, left-padded to
token_len (the host-side branch of the EmbedFromStrings algorithm), for
int32 and int64 widths, with one and several threads, and its argument
checks."""
import numpy as np
import pytest

import oracle
import paper_2601_05531_amd as dt
import synth


def _want(lut, pad_id, rows, T):
    n, L = rows.shape
    offs = np.arange(n + 1, dtype=np.int64) * L
    ids, oo = oracle.encode(oracle.LUT256, rows.reshape(-1), offs, lut=lut)
    w, _ = oracle.pad(ids, oo, T, oracle.LEFT, pad_id)
    return w


@pytest.mark.parametrize("width", [4, 8])
@pytest.mark.parametrize("threads", [1, 3, 16])
def test_map_equals_oracle_table_encode_left_padded(width, threads):
    rng = np.random.default_rng(11)
    data, _ = synth.workload_markov_batch(37, 501)
    rows = data.reshape(37, 501).copy()
    rows.reshape(-1)[rng.integers(0, rows.size, 200)] = rng.integers(0, 256, 200).astype(np.uint8)
    lut = oracle.fallback_lut()
    for T, pad_id in ((501, 0), (777, 0), (512, 9)):
        got = dt.dnatok_ids_map(lut, pad_id, rows, 37, 501, T, width, threads)
        assert got.dtype == (np.int32 if width == 4 else np.int64)
        assert np.array_equal(got.astype(np.int64), _want(lut, pad_id, rows, T).astype(np.int64))


def test_map_single_table_and_large_ids():
    lut = np.arange(256, dtype=np.int32) * 1000003 % 2_000_000_000  # ids beyond 16 bits
    rows = np.arange(4 * 300, dtype=np.int64).astype(np.uint8).reshape(4, 300)
    got = dt.dnatok_ids_map(lut, 7, rows, 4, 300, 301, 8, 2)
    assert np.array_equal(got, _want(lut, 7, rows, 301).astype(np.int64))


def test_map_edge_sizes():
    lut = oracle.fallback_lut()
    assert dt.dnatok_ids_map(lut, 0, np.zeros(0, np.uint8), 0, 5, 5, 4).shape == (0, 5)
    one = np.frombuffer(b"ACGTNacgtnX", dtype=np.uint8).reshape(1, 11)
    assert dt.dnatok_ids_map(lut, 0, one, 1, 11, 11, 4).tolist() == [[1, 2, 3, 4, 0, 1, 2, 3, 4, 0, 0]]
    assert dt.dnatok_ids_map(lut, 5, one, 1, 11, 13, 8).tolist() == [[5, 5, 1, 2, 3, 4, 0, 1, 2, 3, 4, 0, 0]]
    empty_rows = dt.dnatok_ids_map(lut, 3, np.zeros(0, np.uint8), 4, 0, 2, 4)
    assert empty_rows.tolist() == [[3, 3]] * 4


def test_map_rejects_bad_arguments():
    lut = oracle.fallback_lut()
    rows = np.zeros((2, 8), np.uint8)
    for width, T in ((2, 8), (4, 7)):
        with pytest.raises(dt.DnatokError) as e:
            dt.dnatok_ids_map(lut, 0, rows, 2, 8, T, width)
        assert e.value.code == dt.EINVAL
