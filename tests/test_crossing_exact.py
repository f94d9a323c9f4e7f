"""Pins of the exact support-sphere crossing (the surrogate's ground truth):
closed forms of the flat case and the FP64 oracle integrator (CPU)."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests import exact


@pytest.mark.parametrize("c", [1.0, 0.93, 0.6, 0.25, 0.02])
def test_flat_crossing_is_the_chord(c):
    dphi, arc = exact.crossing_exact(0.0, c)
    assert abs(dphi - (np.pi - 2.0 * np.arccos(c))) < 1e-12
    assert abs(arc - 6.0 * c) < 1e-12


def _oracle_crossing(kappa, c, h=2e-3):
    """FP64 RK4 from (3, 0, 0) with g-unit speed until |x| > 3; the exit by
    linear interpolation of |x| between the last two nodes."""
    metric = {"kind": W.GRAPH_GAUSS, "bumps": np.array([[[kappa, 0.0, 0.0, 0.0, 1.0]]], np.float32),
              "twist_amp": 0.0, "twist_theta0": 0.0, "cull_sigmas": 6.0}
    scene = {"spheres": np.zeros((0, 4), np.float32), "planes": np.zeros((0, 4), np.float32),
             "tori": np.zeros((0, 8), np.float32)}
    orc = oracle.Oracle(metric, scene)
    s = np.sqrt(1.0 - c * c)
    x0 = np.array([3.0, 0.0, 0.0])
    d = np.array([-c, s, 0.0])
    g = orc.metric_tensor(x0)
    y0 = d / np.sqrt(d @ g @ d)
    rule = W.rule(kind=W.RK4, h=h, t_max=50.0)
    n = int(8.0 / h)
    traj = orc.trajectory(rule, np.concatenate([x0, y0]), n)
    r = np.linalg.norm(traj[:, :3], axis=1)
    k = int(np.argmax(r[1:] > 3.0)) + 1
    f = (3.0 - r[k - 1]) / (r[k] - r[k - 1])
    xe = traj[k - 1, :3] + f * (traj[k, :3] - traj[k - 1, :3])
    return np.arctan2(xe[1], xe[0]) % (2 * np.pi), (k - 1 + f) * h


@pytest.mark.parametrize("kappa,c", [(0.8, 0.7), (2.0, 0.35), (3.0, 0.9), (1.5, 0.1)])
def test_crossing_matches_oracle_integration(kappa, c):
    dphi, arc = exact.crossing_exact(kappa, c)
    ophi, oarc = _oracle_crossing(kappa, c)
    assert abs(dphi - ophi) < 2e-6, (dphi, ophi)
    assert abs(arc - oarc) < 2e-5, (arc, oarc)


def test_crossing_is_time_reversal_symmetric():
    """Exit direction at polar angle (swept angle + th): the reversed ray
    retraces the path, so the exit makes the entry's angle with the normal."""
    kappa, c = 2.0, 0.5
    metric = {"kind": W.GRAPH_GAUSS, "bumps": np.array([[[kappa, 0.0, 0.0, 0.0, 1.0]]], np.float32),
              "twist_amp": 0.0, "twist_theta0": 0.0, "cull_sigmas": 6.0}
    scene = {"spheres": np.zeros((0, 4), np.float32), "planes": np.zeros((0, 4), np.float32),
             "tori": np.zeros((0, 8), np.float32)}
    orc = oracle.Oracle(metric, scene)
    s = np.sqrt(1 - c * c)
    x0 = np.array([3.0, 0.0, 0.0])
    d = np.array([-c, s, 0.0])
    y0 = d / np.sqrt(d @ orc.metric_tensor(x0) @ d)
    h = 1e-3
    traj = orc.trajectory(W.rule(kind=W.RK4, h=h, t_max=50.0), np.concatenate([x0, y0]), 8000)
    r = np.linalg.norm(traj[:, :3], axis=1)
    k = int(np.argmax(r[1:] > 3.0)) + 1
    f = (3.0 - r[k - 1]) / (r[k] - r[k - 1])
    xe = traj[k - 1] + f * (traj[k] - traj[k - 1])
    phi = np.arctan2(xe[1], xe[0])
    psi = np.arctan2(xe[4], xe[3])
    dphi, _ = exact.crossing_exact(kappa, c)
    assert abs(phi - dphi) < 1e-5
    assert abs(((psi - phi - np.arccos(c)) + np.pi) % (2 * np.pi) - np.pi) < 1e-5
