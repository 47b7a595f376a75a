"""Pins of the oracle's travel-time matrix (Eq (1) of the paper).

The haversine formula is pinned against facts of spherical geometry that do
not go through it: arcs along a meridian and along the equator are R times the
angle, a quarter great circle is pi R / 2, antipodes are pi R apart, the
spherical law of cosines (a different formula) gives the same distance, and
great-circle distance is symmetric, zero on the diagonal and obeys the
triangle inequality.  R = 6371 km, speed 260 km/h, seconds rounded half away
from zero.
"""
import math

import numpy as np
import pytest

import oracle
from gen.instances import SplitMix64, small_instance, m400_instance

R_KM = 6371.0
SPEED = 260.0


def _secs(km):
    return km * 3600.0 / SPEED


def _round_half_away(x):
    return int(math.floor(x + 0.5)) if x >= 0 else -int(math.floor(-x + 0.5))


def _assert_int_close(got, exact_sec):
    """got must be the rounding of exact_sec, unless exact_sec sits within 1e-6 s of a .5 tie."""
    frac = exact_sec - math.floor(exact_sec)
    if abs(frac - 0.5) < 1e-6:
        assert got in (math.floor(exact_sec), math.floor(exact_sec) + 1)
    else:
        assert got == _round_half_away(exact_sec), (got, exact_sec)


def test_one_degree_of_latitude():
    # 1 deg of latitude = 2 pi R / 360 = 111.19492664 km -> 1539.62 s at 260 km/h -> 1540 s
    T = oracle.travel([48.0, 49.0], [-85.0, -85.0], SPEED)
    assert T[0, 1] == 1540 and T[1, 0] == 1540
    assert T[0, 0] == 0 and T[1, 1] == 0


def test_meridian_and_equator_arcs():
    rng = SplitMix64(123)
    for _ in range(200):
        lat1 = -80 + 160 * rng.u01()
        lat2 = -80 + 160 * rng.u01()
        lon = -180 + 360 * rng.u01()
        T = oracle.travel([lat1, lat2], [lon, lon], SPEED)
        _assert_int_close(int(T[0, 1]), _secs(R_KM * abs(math.radians(lat2 - lat1))))
        lon1 = -170 + 340 * rng.u01()
        lon2 = lon1 + (-170 + 340 * rng.u01()) / 2
        T = oracle.travel([0.0, 0.0], [lon1, lon2], SPEED)
        _assert_int_close(int(T[0, 1]), _secs(R_KM * abs(math.radians(lon2 - lon1))))


def test_quarter_circle_and_antipodes():
    T = oracle.travel([0.0, 0.0, 90.0, 0.0], [0.0, 90.0, 0.0, 180.0], SPEED)
    quarter = _secs(math.pi * R_KM / 2)          # 10007.54 km
    half = _secs(math.pi * R_KM)                 # 20015.09 km
    _assert_int_close(int(T[0, 1]), quarter)
    _assert_int_close(int(T[0, 2]), quarter)
    _assert_int_close(int(T[0, 3]), half)
    # over the pole: (phi, 0) to (phi, 180) is R (pi - 2 phi)
    for phi in (10.0, 42.0, 57.0, 75.0):
        T = oracle.travel([phi, phi], [0.0, 180.0], SPEED)
        _assert_int_close(int(T[0, 1]), _secs(R_KM * (math.pi - 2 * math.radians(phi))))


def test_law_of_cosines_agrees_in_the_box():
    inst = m400_instance(0)
    T = oracle.travel(inst.lat, inst.lon, SPEED)
    lat = np.radians(inst.lat)
    lon = np.radians(inst.lon)
    checked = 0
    for i in range(0, inst.n_locs, 7):
        for j in range(inst.n_locs):
            if i == j:
                continue
            c = (math.sin(lat[i]) * math.sin(lat[j])
                 + math.cos(lat[i]) * math.cos(lat[j]) * math.cos(lon[j] - lon[i]))
            km = R_KM * math.acos(max(-1.0, min(1.0, c)))
            if km < 50.0:
                continue   # acos is ill-conditioned for short arcs
            _assert_int_close(int(T[i, j]), _secs(km))
            checked += 1
    assert checked > 2000


@pytest.mark.parametrize("maker", [small_instance, m400_instance])
def test_symmetry_diagonal_triangle(maker):
    inst = maker(0)
    T = oracle.travel(inst.lat, inst.lon, SPEED).astype(np.int64)
    n = T.shape[0]
    assert np.all(np.diag(T) == 0)
    assert np.array_equal(T, T.T)
    assert np.all(T[~np.eye(n, dtype=bool)] > 0)
    # great-circle distance obeys the triangle inequality; each rounding adds <= 0.5 s
    for k in range(0, n, max(1, n // 17)):
        assert np.all(T <= T[:, [k]] + T[[k], :] + 1)
    # the box corners are about 2190 km apart: about 30320 s
    assert T.max() <= 30400


def test_box_extent():
    T = oracle.travel([42.0, 57.0], [-95.0, -75.0], SPEED)
    # corner to corner of the 42-57 N, 75-95 W box
    lat1, lat2 = math.radians(42.0), math.radians(57.0)
    c = (math.sin(lat1) * math.sin(lat2) + math.cos(lat1) * math.cos(lat2)
         * math.cos(math.radians(20.0)))
    _assert_int_close(int(T[0, 1]), _secs(R_KM * math.acos(c)))
