"""Host-side check of the scheme scan's table (no GPU): one line per row, in the given order,
with the exact value, the interval and the error columns."""
from paper_1901_02211_amd.scan import markdown


def _row(r, mode, nsrc, Q, Q_ex):
    return dict(r=r, mode=mode, r_min=float(r), nearest=4, n_classes=nsrc // 12, n_sources=nsrc,
                sources_over_point=nsrc / 3072, Q=Q, abs_dQ=abs(Q - Q_ex), max_abs_dq=0.5, rms_dq=0.25,
                max_abs_imag_q=0.0, seconds=1.0, iterations=10)


def test_markdown_table():
    res = dict(quantity="qx", Q_exact=2.0, n_point_sources=3072, seconds_exact=12.0, interval=(0.15, 2.75),
               rows=[_row(2, 0, 192, 1.5, 2.0), _row(4, 0, 3072, 2.0, 2.0)])
    lines = markdown(res, "flux8").splitlines()
    assert lines[0] == "### flux8"
    assert "Exact Q = 2.000000 from 3072 point sources" in lines[2] and "[0.1500, 2.7500]" in lines[2]
    body = [ln for ln in lines if ln.startswith("| 2 ") or ln.startswith("| 4 ")]
    assert len(body) == 2 and "| 192 |" in body[0] and "5.00e-01" in body[0] and "0.00e+00" in body[1]


def test_markdown_trace_of_inverse_has_no_interval():
    res = dict(quantity="trinv", Q_exact=10.0, n_point_sources=3072, seconds_exact=1.0, interval=(None, None),
               rows=[])
    text = markdown(res, "t")
    assert "Exact Tr D_W^-1 = 10.000000" in text and "Zolotarev" not in text
