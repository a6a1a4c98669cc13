"""Pins for the oracle's concrete renderer (Alg. GaussianSplat, BlendSort, BlendInd)."""
import itertools

import numpy as np
import pytest

from oracle import render
from paper_2503_00308_amd import synth

RNG = np.random.default_rng(99)


def test_lemma_blendsort_equals_blendind_distinct_depths():
    """Lemma 'sort-to-ind' on random concrete inputs with distinct depths."""
    for n in (1, 2, 5, 17, 60):
        a = RNG.uniform(0, 1, (n, 33))
        c = RNG.uniform(0, 1, (n, 3))
        d = RNG.permutation(n).astype(float) + RNG.uniform(0, 0.5, n)
        np.testing.assert_allclose(render.blend_sort(a, c, d), render.blend_ind(a, c, d), rtol=1e-12, atol=1e-14)


def test_blend_ties_share_transmittance():
    """With equal depths Ind(0) = 0: tied Gaussians do not occlude each other (both blends agree)."""
    a = RNG.uniform(0, 1, (6, 5))
    c = RNG.uniform(0, 1, (6, 3))
    d = np.array([1.0, 2.0, 2.0, 3.0, 2.0, 0.5])
    np.testing.assert_allclose(render.blend_sort(a, c, d), render.blend_ind(a, c, d), rtol=1e-12)


def test_blendsort_matches_textbook_front_to_back():
    """Front-to-back compositing C += T a c, T *= (1 - a) in depth order (distinct depths)."""
    n = 8
    a = RNG.uniform(0, 1, (n, 4))
    c = RNG.uniform(0, 1, (n, 3))
    d = RNG.permutation(n).astype(float)
    C = np.zeros((4, 3))
    T = np.ones(4)
    for i in np.argsort(d):
        C += (T * a[i])[:, None] * c[i][None, :]
        T *= 1 - a[i]
    np.testing.assert_allclose(render.blend_sort(a, c, d), C, rtol=1e-13)


def test_alpha_matches_projected_gaussian_density():
    """The q and a steps give o exp(-1/2 (u-mu)^T S^-1 (u-mu)) with S the projected covariance.

    Reference computed independently: mu = (fx x/z, fy y/z), S = G Cov_c G^T with the
    perspective Jacobian G = [[fx/z, 0, -fx x/z^2], [0, fy/z, -fy y/z^2]].
    """
    sc = synth.random_scene(40, seed=3)
    intr = synth.intrinsics(48)
    box = synth.camera6_box()
    R, t = np.eye(3), np.zeros(3)
    proj = render.project(sc, intr, R, t)
    ux, uy = render.pixel_grid(intr)
    a = render.alpha(sc, intr, proj, ux, uy, 0.01)
    uw = sc["mean"].astype(np.float64)
    for i in range(len(uw)):
        x, y, z = uw[i]
        G = np.array([[intr["fx"] / z, 0, -intr["fx"] * x / z ** 2], [0, intr["fy"] / z, -intr["fy"] * y / z ** 2]])
        M = sc["cov_factor"][i].astype(np.float64)
        S = G @ (M @ M.T) @ G.T
        mu = np.array([intr["fx"] * x / z, intr["fy"] * y / z])
        du = np.stack([ux - mu[0], uy - mu[1]], axis=1)
        m2 = np.einsum("pi,ij,pj->p", du, np.linalg.inv(S), du)
        ref = sc["opacity"][i] * np.exp(-0.5 * m2)
        np.testing.assert_allclose(a[i], ref, rtol=1e-9, atol=1e-300)


def test_render_single_gaussian_peak():
    """One Gaussian on the optical axis: the centre pixel gets colour o * c exactly."""
    sc = {"mean": np.array([[0.0, 0.0, 4.0]], np.float32),
          "cov_factor": (0.1 * np.eye(3))[None].astype(np.float32),
          "opacity": np.array([0.7], np.float32), "rgb": np.array([[0.2, 0.5, 1.0]], np.float32)}
    intr = {"width": 3, "height": 3, "fx": 3.0, "fy": 3.0, "cx": 1.5, "cy": 1.5}
    img = render.render(sc, intr, synth.camera6_box(), np.zeros(6))
    np.testing.assert_allclose(img[1, 1], 0.7 * np.array([0.2, 0.5, 1.0]), rtol=1e-6)


def test_near_plane_and_behind_camera():
    sc = {"mean": np.array([[0.0, 0.0, -1.0], [0.0, 0.0, 0.005]], np.float32),
          "cov_factor": np.stack([0.1 * np.eye(3)] * 2).astype(np.float32),
          "opacity": np.array([0.9, 0.9], np.float32), "rgb": np.ones((2, 3), np.float32)}
    intr = synth.intrinsics(8)
    img = render.render(sc, intr, synth.camera6_box(), np.zeros(6))
    assert np.all(img == 0)


def test_camera_translation_moves_image():
    """Translating the camera by +dx shifts a Gaussian's projection by -fx dx / z."""
    sc = {"mean": np.array([[0.0, 0.0, 4.0]], np.float32),
          "cov_factor": (0.05 * np.eye(3))[None].astype(np.float32),
          "opacity": np.array([0.9], np.float32), "rgb": np.ones((1, 3), np.float32)}
    intr = synth.intrinsics(64)
    box = synth.camera6_box(dt=(0.5, 0, 0))
    img = render.render(sc, intr, box, np.array([0.5, 0, 0, 0, 0, 0]))
    col = np.argmax(img[32, :, 0])
    expected = 32 - 64 * 0.5 / 4.0
    assert abs((col + 0.5) - expected) <= 1.0
