"""Pins for the operation-count model against the paper's printed leading orders."""
from oracle import flops


def test_quadrature_ratios_at_feorder_8():
    np_ = 9
    base = flops.flop_mf_real(np_, np_, 1, 1)
    r2 = flops.flop_mf_real(np_, np_ + 2, 1, 1) / base
    r3 = flops.flop_mf_real(np_, np_ + 3, 1, 1) / flops.flop_mf_real(np_, np_ + 2, 1, 1)
    assert abs(r2 - 1.8) < 0.1       # "about 1.8x" fewer when lowering n_p+2 -> n_p
    assert abs(r3 - 1.4) < 0.05      # "about 1.4x" more when raising n_p+2 -> n_p+3


def test_leading_orders():
    for np_ in (7, 8, 9, 10):
        mf = flops.flop_mf_real(np_, np_, 1, 1)
        assert 0.7 < mf / (12 * np_ ** 4) < 2.0
        assert flops.flop_cm_real(np_, 1, 1) == 2 * np_ ** 6
        assert flops.flop_cm_complex(np_, 1, 1) == 6 * np_ ** 6
        assert flops.flop_mf_complex(np_, np_, 1, 1) > 2 * mf
