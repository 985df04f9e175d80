"""Whole-loop pins: noise-free convergence to the known object up to a global
phase (ePIE's fixed point), and the paper's qualitative claim that the
Gaussian convolution of box 1 helps on blurred data (Sec. 3.1, Figs. 3-4)."""

import numpy as np

import datagen
import oracle as ora


def _small(sigma_data):
    spec = dict(datagen.CONFIGS["far64"])
    spec.update(obj=(64, 64), n=32, n_side=5, step=6, radius=9, jitter=1, sigma_data=sigma_data)
    return spec, datagen.make_scan(spec, 7, noise=False, probe_known=True)


def test_coherent_noise_free_converges_to_truth():
    spec, s = _small(0.0)
    roi = ora.illumination_roi(s["positions"], s["probe_true"], spec["obj"], 0.3)
    params = ora.Params(n=32, sigma1=0.0, sigma2=0.0, probe_update_start=10 ** 6, eps=1e-9)
    st, errs = ora.iterate(ora.State(O=s["obj0"], P=s["probe0"]), s["intensities"],
                           s["positions"], params, 40)
    assert ora.nmse(st.O, s["obj_true"], roi) < 1e-8
    assert errs[-1] < 1e-8


def test_gaussian_convolution_beats_plain_epie_on_blurred_data():
    spec, s = _small(1.0)
    roi = ora.illumination_roi(s["positions"], s["probe_true"], spec["obj"], 0.3)
    res = {}
    for sig in (0.0, 1.0):
        params = ora.Params(n=32, sigma1=sig, sigma2=sig, probe_update_start=10 ** 6)
        st, errs = ora.iterate(ora.State(O=s["obj0"], P=s["probe0"]), s["intensities"],
                               s["positions"], params, 20)
        res[sig] = (ora.nmse(st.O, s["obj_true"], roi), errs[-1])
    assert res[1.0][0] < 0.25 * res[0.0][0]
    assert res[1.0][1] < 0.25 * res[0.0][1]
