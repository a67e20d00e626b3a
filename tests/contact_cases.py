"""Seeded contact scenes shared by the CPU and GPU contact tests: systems,
contact spheres (links, centres in link coordinates, radii), initial states
and controls.  Geometry and random draws only."""
import numpy as np

from paper_2109_07719_amd import synth


def landing_quadruped(seed, T, drop=0.005):
    return synth.landing_quadruped(seed, T, drop)


def grounded_tree(seed, T, rng_seed=None):
    """A fixed-base tree with prismatic joints and random frames, four
    spheres on random links, the root lowered so that every sphere starts
    1-5 mm below the ground plane."""
    rng = np.random.default_rng(seed if rng_seed is None else rng_seed)
    s, q0, qd0, tau = synth.tree_system(seed, T, nmin=6, nmax=12, random_frames=True, prismatic=0.3)
    k = 4
    links = np.sort(rng.choice(np.arange(1, s.n), size=k, replace=False)).astype(np.int32)
    centers = rng.normal(0, 0.15, (k, 3))
    radii = rng.uniform(0.03, 0.08, k)
    return s, q0, qd0, tau, links, centers, radii


def lower_to_ground(s, q0, links, centers, radii, world_points, depth):
    """Shift the root's placement so that the highest sphere bottom sits at
    -depth (every sphere starts in contact)."""
    ys = [world_points(s, q0, l, c)[1] - r for l, c, r in zip(links, centers, radii)]
    s.r_T[0] = s.r_T[0] - np.array([0.0, max(ys) + depth, 0.0])
    return s


def resting_chain(T, seed=5):
    """A planar 3-link chain lying along x on the ground with spheres on link
    1's middle and link 2's tip sunk 2 mm (persistent contact)."""
    s, _, _, _ = synth.chain_system(3, 7, T)
    s.r_T[0] = [0.0, 0.05 - 2e-3, 0.0]
    rng = np.random.default_rng(seed)
    q0 = rng.normal(0, 1e-3, 3)
    qd0 = rng.normal(0, 1e-3, 3)
    tau = rng.normal(0, 0.5, (T, 3))
    return s, q0, qd0, tau, np.array([1, 2], np.int32), np.array([[0.25, 0.0, 0.0], [0.5, 0.0, 0.0]]), np.full(2, 0.05)
