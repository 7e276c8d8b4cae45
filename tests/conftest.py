import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.lib()
    return oracle


def make_scene(pos, nrm, tan, scl, alb=None, rough=None, metal=None, envmap=None):
    """A scene from per-surfel rows ([N][3] style arrays are transposed to [C][N])."""
    from scenegen import Scene
    f = lambda a: np.ascontiguousarray(np.asarray(a, np.float64).T, np.float32)
    pos = np.atleast_2d(pos)
    n = pos.shape[0]
    if alb is None:
        alb = np.full((n, 3), 0.5)
    if rough is None:
        rough = np.full(n, 0.5)
    if metal is None:
        metal = np.zeros(n)
    return Scene(f(pos), f(np.atleast_2d(nrm)), f(np.atleast_2d(tan)), f(np.atleast_2d(scl)),
                 f(np.atleast_2d(alb)), np.asarray(rough, np.float32), np.asarray(metal, np.float32),
                 envmap)


def axis_camera(w=64, h=64, f=100.0, R=None, t=None, background=(0.0, 0.0, 0.0)):
    """Pinhole camera at the origin looking down +z (or R, t if given)."""
    from scenegen import Camera
    R = np.eye(3, dtype=np.float32) if R is None else np.asarray(R, np.float32)
    t = np.zeros(3, np.float32) if t is None else np.asarray(t, np.float32)
    return Camera(w, h, f, f, w / 2.0, h / 2.0, R, t, 0.01, tuple(background), 0)
