import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU-only oracle runs")


def pytest_addoption(parser):
    parser.addoption("--runslow", action="store_true", default=False,
                     help="also run the long CPU-only oracle runs marked slow")


def pytest_collection_modifyitems(config, items):
    if config.getoption("--runslow") or os.environ.get("IPC_RUN_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="long oracle run: use --runslow")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    return oracle.lib()


@pytest.fixture(scope="session")
def c1_oracle_trajectory():
    """Oracle iterates of config 1: per step, (x^t, v^t, pose, [x_k])."""
    import oracle
    from paper_2411_04776_amd import scenes
    sc = scenes.config1()
    o = oracle.OracleScene(sc)
    traj = []
    for step in range(1, sc.n_steps + 1):
        pose = sc.poses[step]
        x0, v0 = o.x, o.v
        o.begin_step(pose)
        xs = [x0]
        x = x0
        for _ in range(100):
            r, xn, st = o.newton_iterate(x)
            if r != 0:
                break
            xs.append(xn)
            x = xn
        traj.append((x0, v0, pose, xs))
        o.step(pose)  # commit exactly as the oracle step does (same iterates)
        assert np.array_equal(o.x, xs[-1])
    return sc, traj, o.x
