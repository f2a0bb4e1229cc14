"""Microbenchmarks of the roofline denominators (needs an MI355X): the
measured VALU issue rate, LDS read and HBM read bandwidth lie between a
floor that only a broken measurement misses and a little above the chip's
published or derived figures (256 CUs x 64 lanes x 2.4 GHz for VALU; 8 TB/s
HBM; 128-256 B per clock per CU for LDS)."""
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_measured_peaks_are_plausible():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_08123_amd as gga
    pk = gga.measure_peaks(1 << 30)
    print(pk)
    valu, lds, hbm = pk["valu_lane_ops_per_s"], pk["lds_read_bytes_per_s"], pk["hbm_read_bytes_per_s"]
    assert 0.5 * 39.32e12 < valu < 1.05 * 39.32e12
    assert 1e12 < hbm < 8.4e12
    assert 20e12 < lds < 1.05 * 256 * 256 * 2.4e9
