"""The measured arithmetic peak (vlp_measure_modmul_peak): rates are
plausible for the instruction count of a butterfly, the CMux mix lies
between its two parts, and a bad device is an argument error."""
import pytest

pytestmark = pytest.mark.gpu


def test_measured_butterfly_rates():
    from paper_2506_12761_amd import vlp
    r = vlp.vlp_measure_modmul_peak(0)
    lane_ops = 256 * 64 * 2.4e9  # VALU lane operations per second at the peak clock
    for k in ("fwd", "inv"):
        # a butterfly is at least 8 VALU instructions (Shoup product, add, subtract, min)
        # and the chip issues at most two per lane and clock
        assert lane_ops / 100 < r[k] < 2 * lane_ops / 8, r
    assert min(r["fwd"], r["inv"]) <= r["mixed"] <= max(r["fwd"], r["inv"])


def test_bad_device_is_rejected():
    from paper_2506_12761_amd import vlp
    with pytest.raises(vlp.VlpError) as e:
        vlp.vlp_measure_modmul_peak(4096)
    assert e.value.status == vlp.VLP_EINVAL
