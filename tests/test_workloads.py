"""The input builders: every mesh they produce is consistent (face
relations symmetric, matched flux points with opposite area normals and
positions differing by one vector per face), so the library accepts it and
the oracle and library see the same mesh."""
import numpy as np
import pytest

import workloads as W


def _face_map(n, o, a, b):
    x, y = (b, a) if o & 1 else (a, b)
    if o & 2:
        x = n - 1 - x
    if o & 4:
        y = n - 1 - y
    return x, y


def _check(orc, mesh, p=2):
    g = orc.geometry(mesh, p)
    n = p + 1
    nf, ne = g["nf"], mesh["n_elem"]
    for e in range(ne):
        for f in range(6):
            nb = mesh["nbr_elem"][e, f]
            if nb < 0:
                assert mesh["bc"][e, f] in (1, 2, 3)
                continue
            fb, o = mesh["nbr_face"][e, f], mesh["nbr_orient"][e, f]
            assert mesh["nbr_elem"][nb, fb] == e and mesh["nbr_face"][nb, fb] == f
            for b in range(n):
                for a in range(n):
                    pa, pb = _face_map(n, o, a, b)
                    u, v = nf[e, f, a + n * b], nf[nb, fb, pa + n * pb]
                    assert np.abs(u + v).max() <= 1e-9 * np.abs(u).max()


@pytest.mark.parametrize("name", ["box", "reoriented", "quadratic", "cylinder", "half_cylinder"])
def test_mesh_builders_are_consistent(orc, name):
    mesh = {"box": lambda: W.box_mesh((3, 2, 2), length=(1.0, 0.8, 0.6)),
            "reoriented": lambda: W.reorient_elements(W.box_mesh((3, 3, 2)), seed=4)[0],
            "quadratic": lambda: W.quadratic_map_mesh((2, 3, 2), eps=0.2),
            "cylinder": lambda: W.cylinder_mesh(n_theta=8, n_r=3, n_z=2, r1=2.0),
            "half_cylinder": lambda: W.cylinder_mesh(n_theta=6, n_r=3, n_z=2, r1=2.0, half=True)}[name]()
    _check(orc, mesh)


def test_paper_freestream_units():
    """Unit speed at angle alpha, theta = P = 1/(gamma M^2), so the speed of
    sound is 1/M; mu = mu_ref = 1/Re at the reference temperature."""
    par = W.paper_freestream(8.0, 5.5e5, 18.5)
    U = np.array(par["farfield"][1:4])
    assert np.linalg.norm(U) == pytest.approx(1.0, abs=1e-15)
    assert np.linalg.norm(U) / np.sqrt(5.0 / 3.0 * par["farfield"][4]) == pytest.approx(8.0, rel=1e-14)
    assert par["mu_ref"] * 5.5e5 == pytest.approx(1.0) and par["theta_ref"] == par["farfield"][4]
