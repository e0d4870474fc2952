"""Host side of the file-backed trajectory store (paper_1511_06959_amd.offload._FileStore): every
record written through a staging buffer in parallel slices reads back byte for byte, through the
staging buffers and directly, whatever the record size (slices that do not divide it, records
smaller than a page).  No GPU: unpinned staging buffers, host events."""
import numpy as np
import pytest
import torch

from paper_1511_06959_amd.offload import _FileStore


class _Done:
    def synchronize(self):
        pass


@pytest.mark.parametrize("rec_len,dtype,io_threads", [(5 * 1000, torch.float64, 4), (12345, torch.uint8, 3),
                                                      (7, torch.float32, 4), (3 * 4096 + 5, torch.float32, 1)])
def test_file_store_round_trip(tmp_path, rec_len, dtype, io_threads):
    n = 5
    path = str(tmp_path / "t.bin")
    st = _FileStore(n, rec_len, dtype, path, nstage=2, io_threads=io_threads, pin=False)
    assert sum(ln for _, ln in st.slices) == st.rec_bytes
    assert all(o % 4096 == 0 for o, _ in st.slices)
    rng = np.random.default_rng(7)
    recs = []
    for k in range(n):
        a = rng.integers(0, 256, size=rec_len * st.stage[0].element_size(), dtype=np.uint8)
        recs.append(a)
        j = st._slot(k)
        st._claim(j)
        st.stage[j].numpy().view(np.uint8)[:] = a
        st.busy[j] = st.pool.submit(st._write, k, j, _Done())
    st.finish()
    import os
    assert os.path.getsize(path) == n * st.rec_bytes
    for k in (3, 0, 4, 1, 2):
        assert np.array_equal(st.read(k).numpy().view(np.uint8), recs[k])
        j = st._slot(k)
        st.stage[j].zero_()
        st._read(k, j, None)
        assert np.array_equal(st.stage[j].numpy().view(np.uint8), recs[k])
    st.close()
    assert not os.path.exists(path)
