"""The oracle's batch clustering search against its pins (cluster_pins.py), and
planted mistakes in copies of oracle/cluster.py that the pins must catch."""
import importlib.util
import os

import pytest

import oracle.cluster
from cluster_pins import ALL_CLUSTER_PINS


@pytest.mark.parametrize("pin", ALL_CLUSTER_PINS, ids=[p.__name__ for p in ALL_CLUSTER_PINS])
def test_cluster_pin(pin):
    pin(oracle.cluster)


MUTATIONS = {
    "majority_ties_up": ("pack_bits(2 * counts > len(members))",
                         "pack_bits(2 * counts >= len(members))"),
    "nearest_is_farthest": ("new = np.argmin(dc, axis=1)", "new = np.argmax(dc, axis=1)"),
    "init_nearest": ("far = int(np.argmax(near))", "far = int(np.argmin(near[1:])) + 1"),
    "silhouette_sign": ("s[i] = (b - a) / top", "s[i] = (a - b) / top"),
    "a_includes_self": ("a = float(sums[own]) / float(size[own] - 1)",
                        "a = float(sums[own]) / float(size[own])"),
    "b_largest": ("b = m if b is None or m < b else b", "b = m if b is None or m > b else b"),
    "no_iteration": ("if not changed:\n            break", "break"),
    "ties_to_larger_k": ("if best is None or sc > best[0]:", "if best is None or sc >= best[0]:"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_cluster_pins_catch_mutation(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(oracle.cluster.__file__).read()
    assert src.count(old) == 1, name
    path = os.path.join(tmp_path, f"cluster_{name}.py")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    spec = importlib.util.spec_from_file_location(f"cluster_{name}", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    failed = []
    for pin in ALL_CLUSTER_PINS:
        try:
            pin(mod)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"no pin catches the planted mistake {name}"
