"""Input generators: the torch evaluation of the sphere's Fourier fields equals
the numpy one; the balanced flow has the stated amplitudes and is in linear
balance (h = f psi / g with u = n x grad psi)."""
import numpy as np

import hdg_inputs as hi


def test_sphere_fields_torch_equals_numpy():
    m = hi.icosphere(2, 6.371e6)
    a = hi.smooth_rhs_sphere(m, 2, 5, nrhs=2)
    b = hi.smooth_rhs_sphere(m, 2, 5, nrhs=2, device="cpu")
    assert np.abs(a - b).max() < 1e-10 * np.abs(a).max()
    assert abs(np.abs(a[:, 0]).max() - 100.0) < 1e-9
    assert abs(np.sqrt(a[:, 1] ** 2 + a[:, 2] ** 2).max() - 20.0) < 1e-9


def test_balanced_flow_amplitudes_and_balance():
    m = hi.icosphere(3, 6.371e6)
    q = hi.balanced_flow_sphere(m, 2, 300, 7.292e-5, 9.81)
    qt = hi.balanced_flow_sphere(m, 2, 300, 7.292e-5, 9.81, device="cpu")
    assert np.abs(q - qt).max() < 1e-10 * np.abs(q).max()
    speed = np.sqrt(q[:, 1] ** 2 + q[:, 2] ** 2)
    assert speed.max() <= 20.0 + 1e-9 and speed.max() > 19.0        # in-plane part of |u| = 20 m/s
    assert 30.0 < np.abs(q[:, 0]).max() < 300.0                        # h ~ 100 m
    # h vanishes on the equator (f = 0 there) and changes sign with the hemisphere
    x = hi.rhs.node_coords(m, 2)
    z = x[..., 2] / np.linalg.norm(x, axis=-1)
    eq = np.abs(z) < 0.02
    assert np.abs(q[:, 0][eq]).max() < 0.1 * np.abs(q[:, 0]).max()
