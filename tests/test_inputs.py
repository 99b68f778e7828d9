"""Host checks of the seeded input generators for the paper's crosswell
example (Numerical Examples: geometry, lens model, bandpass wavelet)."""
import numpy as np

import inputs


def test_bandpass_wavelet_spectrum_and_centre():
    dt = 1e-3
    t = np.arange(8192) * dt
    w = inputs.bandpass_wavelet(t, t0=2.0)
    assert abs(t[np.argmax(w)] - 2.0) < 2 * dt and abs(w.max() - 1.0) < 1e-2
    amp = np.abs(np.fft.rfft(w))
    f = np.fft.rfftfreq(t.size, dt)
    a = lambda fr: amp[np.argmin(np.abs(f - fr))] / amp.max()  # noqa: E731
    # flat pass band, half height halfway up each ramp, nothing outside
    assert min(a(3.0), a(5.0), a(7.0)) > 0.97
    assert abs(a(1.75) - 0.5) < 0.05 and abs(a(10.0) - 0.5) < 0.05
    assert a(0.5) < 0.02 and a(14.0) < 0.02


def test_crosswell_geometry():
    prob = inputs.crosswell_problem()
    assert (prob.nz, prob.nx, prob.h) == (201, 401, 20.0)
    assert (prob.z_src, prob.z_rec) == (3000.0, 1000.0)
    assert prob.x_src0 == prob.x_rec0 == 2000.0 and prob.ns == prob.nr == 201
    assert prob.slab_dz == prob.rslab_dz == -5 and prob.xs == (3500.0,)
    kap = inputs.crosswell_kappa()
    assert kap.shape == (201, 401)
    assert abs(kap[100, 200] - 1.6e9) < 1.0 and abs(kap[0, 0] - 4.0e9) < 1e3
    assert np.all(inputs.crosswell_kappa(lens=False) == 4.0e9)
    pt = inputs.crosswell_point_problem(prob)
    assert (pt.z_src, pt.x_src0, pt.ns) == (3500.0, 3500.0, 1)
