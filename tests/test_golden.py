"""Pins against values the paper prints (fixtures under tests/golden/, each citing its
passage): the Eq. 16/17 mask and constant, the pupil pre-filter of Algorithm 1, and the
Eq. 19 defaults.  The oracle is checked against brute-force evaluations built from the
fixtures, not against its own constants."""
import math
import os

import numpy as np

import oracle as orc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_fixture(name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            rows.setdefault(key, []).append(vals)
    return rows


def test_penalty_weight_matches_printed_mask_and_constant():
    f = read_fixture("eq16_17_penalty.txt")
    mask = np.array([[float(v) for v in r] for r in f["mask_row"]])
    assert f["c_sqrt"][0][0] == "pi/2"
    c = float(f["c_num"][0][0]) / float(f["c_den"][0][0]) * math.sqrt(math.pi / 2)
    rng = np.random.default_rng(16)
    stack = rng.random((3, 7, 6)) * 4.0
    for fid, g in ((orc.FID_INTENSITY, lambda x: x), (orc.FID_AMPLITUDE, np.sqrt)):
        total = 0.0
        for img in g(stack):
            H, W = img.shape
            for y in range(1, H - 1):  # positions where the mask fits
                for x in range(1, W - 1):
                    acc = 0.0
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            acc += mask[1 - dy, 1 - dx] * img[y + dy, x + dx]  # convolution
                    total += abs(acc) / (W * H)
        want = c * total / stack.shape[0]
        assert abs(orc.auto_penalty(stack, fid) - want) < 1e-12 * want


def test_pupil_prefilter_is_the_printed_gaussian():
    f = read_fixture("alg1_pupil_prefilter.txt")
    size, sigma = int(f["size"][0][0]), float(f["sigma_px"][0][0])
    h = size // 2
    w = np.array([[math.exp(-(dx * dx + dy * dy) / (2 * sigma * sigma)) for dx in range(-h, h + 1)]
                  for dy in range(-h, h + 1)])
    w /= w.sum()
    assert orc.gauss3_weights().shape == (size, size)
    assert np.allclose(orc.gauss3_weights(), w, rtol=0, atol=1e-15)


def test_adabelief_defaults_are_the_printed_ones():
    f = read_fixture("eq19_defaults.txt")
    g1, g2 = float(f["gamma1"][0][0]), float(f["gamma2"][0][0])
    prob = orc.Problem(n_lo=8, upsample=2, led_k=np.zeros((1, 2)), wavelength_um=0.5, na=0.1, dx_lo_um=1.0)
    assert (prob.gamma1, prob.gamma2) == (g1, g2)
    st = orc.new_state(np.ones((16, 16), complex), np.ones((8, 8), complex), prob)
    assert float(f["mu0"][0][0]) == 0.0 and not st.mu_psi.any() and not st.mu_P.any()
    assert float(f["v0"][0][0]) == 0.0 and not st.v_psi.any() and not st.v_P.any()
