"""Host logic of the learned-guess training (no GPU): the crop of a large
mesh around a stimulus site used to train on trajectories of the 17M-dof
slab."""
import numpy as np

from paper_2101_02959_amd.predictor import crop_nodes
from workload import Mesh, stimulus_nodal


def test_crop_nodes_is_a_lexicographic_box_containing_the_site():
    m = Mesh(40, 30, 20, 0.01, (0, 20, 40), (0, 15, 30), (0, 10, 20))
    for origin in [(0, 0, 0), (38, 28, 18), (17, 5, 9)]:
        idx = crop_nodes(m, origin, (2, 2, 2), 9)
        assert idx.size == 9 ** 3 and np.unique(idx).size == idx.size
        i = idx % (m.nx + 1)
        j = (idx // (m.nx + 1)) % (m.ny + 1)
        k = idx // ((m.nx + 1) * (m.ny + 1))
        assert i.min() >= 0 and i.max() <= m.nx and j.max() <= m.ny and k.max() <= m.nz
        # x fastest, then y, then z: the crop is itself a lexicographic grid
        g = np.stack([k, j, i], axis=1).reshape(9, 9, 9, 3)
        assert np.all(np.diff(g[..., 2], axis=2) == 1)
        assert np.all(np.diff(g[..., 1], axis=1) == 1)
        assert np.all(np.diff(g[..., 0], axis=0) == 1)
        # every stimulated node lies in the crop
        stim = np.nonzero(stimulus_nodal(m, (2, 2, 2), 1.0, origin))[0]
        assert np.isin(stim, idx).all()
