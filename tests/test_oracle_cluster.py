"""Cluster cuts of a periodic structure (the sampled-atom checks on systems
too large for the oracle rely on them).  Locality of the method (Section 2.1:
every atomic energy sums over neighbours within the cutoff): an atom's energy
depends only on atoms within r_c, its force only on atoms within 2 r_c, so a
non-periodic cluster of radius R reproduces the periodic energies within
R - r_c of its centre and the periodic forces within R - 2 r_c."""
import numpy as np

from oracle import brute_force_neighbors, evaluate
from workloads import cluster_cut, make_workload


def test_cluster_reproduces_periodic_energies_and_forces():
    batch, params, spec = make_workload("solid", reps=(11, 11, 11))  # 25.5 A box
    rc = spec.model.r_cut
    full = evaluate(batch, params, brute_force_neighbors(batch, rc), want_stress=False)
    R = 2 * rc + 0.5
    for center in (0, 777):
        cut, idx, dist = cluster_cut(batch, center, R)
        assert idx[0] == center and dist[0] == 0.0
        assert cut.pbc.sum() == 0 and np.all(dist < R)
        sub = evaluate(cut, params, brute_force_neighbors(cut, rc), want_stress=False)
        inner_f = dist < R - 2 * rc
        inner_e = dist < R - rc
        assert inner_f.sum() >= 1 and inner_e.sum() > 20
        assert np.abs(sub.forces[inner_f] - full.forces[idx[inner_f]]).max() < 1e-10
        assert np.abs(sub.atomic[inner_e] - full.atomic[idx[inner_e]]).max() < 1e-10
        # atoms near the cluster's surface miss neighbours: their energies differ
        outer = dist > R - 1.0
        assert np.abs(sub.atomic[outer] - full.atomic[idx[outer]]).max() > 1e-3
