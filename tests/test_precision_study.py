"""CPU check of the precision study (tests/precision_study.py) on a few cells:
the orderings behind the design of the mixed path hold, and the packing of two
directions into one complex transform is exact."""

import os
import sys

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import precision_study as ps  # noqa: E402


def test_2d_orderings():
    r = ps.study_2d(4)
    err = {k: v[0] for k, v in r.items()}
    assert err["packing_exact"] < 1e-11
    # FP32 intermediates cap the accuracy near 1e-5 whatever the GEMMs do ...
    assert err["exact_f32"] > 3e-6 and err["fp32_mfma"] > 1e-5 and err["fp16x3_f32"] > 1e-5
    # ... the fixed-point-lead split with FP64 intermediates clears 1e-5, and FP64
    # filters gain another order of magnitude
    assert err["fx16"] < 1e-6 < err["fx16_f32filt"] < 1e-5
    assert err["fx16"] * 5 < err["fx16_f32filt"] < err["exact_f32"] < err["fp32_mfma"]
    # each of the six FP16 products is needed: without the data's lo part the
    # error is far above 1e-5, without the DFT matrix's lo part an order of
    # magnitude above the full split's
    assert err["fx16_no_lo_data"] > 1e-4 and err["fx16_no_lo_dft"] > 10 * err["fx16"]
