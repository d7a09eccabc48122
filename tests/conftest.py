import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library on the device)")


def rot_angle(Ra, Rb):
    """Angle of Ra Rb^T in radians, atan2 form (accurate for tiny angles)."""
    M = np.asarray(Ra) @ np.asarray(Rb).T
    s = 0.5 * np.array([M[2, 1] - M[1, 2], M[0, 2] - M[2, 0], M[1, 0] - M[0, 1]])
    return float(np.arctan2(np.linalg.norm(s), 0.5 * (np.trace(M) - 1.0)))


def pose_close(Ra, ta, Rb, tb, deg=1e-3, rel_t=1e-4):
    """Final-pose tolerance: angle within `deg` degrees and
    |ta - tb| <= rel_t * max(|tb|, 1 m)."""
    ang = np.degrees(rot_angle(Ra, Rb))
    dt = float(np.linalg.norm(np.asarray(ta) - np.asarray(tb)))
    return ang <= deg and dt <= rel_t * max(float(np.linalg.norm(tb)), 1.0), ang, dt


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle
