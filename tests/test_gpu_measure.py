"""gb_lds_peak, the measurement behind the bench's LDS roofline: positive,
plausible rates for both read widths (16-byte reads move at least as many
bytes per second as 4-byte ones, and neither exceeds 512 bytes per CU per
clock at 3 GHz), and GB_EINVAL for another width."""
import pytest

pytestmark = pytest.mark.gpu


def test_lds_peak():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2603_07850_amd as gb
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    print("[gpu-measure] gb_lds_peak on %d CUs" % cus, flush=True)
    r16, r4 = gb.lds_peak(16), gb.lds_peak(4)
    ceiling = 512.0 * cus * 3e9
    assert 0 < r4 <= r16 * 1.05 and r16 < ceiling, (r4, r16)
    with pytest.raises(gb.GoldbachError) as e:
        gb.lds_peak(8)
    assert e.value.name == "GB_EINVAL"
