"""Host-side bounds check of the fused plane kernels' launch geometry (no GPU).

Restates, in NumPy, the index arithmetic of the plane kernels and their launch as the
library writes it: the coil-group choice at plan creation (largest group up to 16 coils, in
either kernel, that still gives every compute unit a workgroup), the grid of n2 * ngroups
workgroups, the XCD-aware workgroup -> (plane i2, coil group) map, the coil range of a group,
and the offsets of every per-(coil, plane) and per-(group, plane) block the kernels read or
write.  Checks that every block lies inside the buffer the plan sizes for it and that each
(plane, group) pair is visited exactly once.
"""
import numpy as np
import pytest

NXCD = 8


def pick(gmax, n2, J, cus=256):
    G = gmax
    while G > 1 and n2 * ((J + G - 1) // G) < cus:
        G //= 2
    return G


def plane_block(ngrp, n2):
    nb = ngrp * n2
    l = np.arange(nb)
    if nb % NXCD == 0:
        l = (l % NXCD) * (nb // NXCD) + l // NXCD
    return l // ngrp, l % ngrp


@pytest.mark.parametrize("n0,n1,n2,r0,r1,J,L", [
    (128, 128, 128, 40, 40, 32, 2048),      # the 128^3, 32-coil workload
    (128, 128, 64, 40, 40, 5, 2048),
    (48, 32, 20, 9, 13, 5, 460),
    (16, 80, 12, 3, 17, 3, 256),
    (32, 32, 16, 9, 10, 64, 307),
    (128, 128, 128, 40, 40, 1, 2048),
    (128, 128, 256, 48, 48, 64, 4096),
])
def test_plane_kernel_blocks_stay_in_their_buffers(n0, n1, n2, r0, r1, J, L):
    N = n0 * n1 * n2
    for kernel, gmax in (("fwd", 16), ("adj", 16)):
        G = pick(gmax, n2, J)
        G_adj = pick(16, n2, J)
        ngrp = (J + G - 1) // G
        i2, gi = plane_block(ngrp, n2)
        # every (plane, group) pair exactly once
        pairs = i2 * ngrp + gi
        assert np.array_equal(np.sort(pairs), np.arange(ngrp * n2))
        assert i2.min() >= 0 and i2.max() < n2
        for w in range(i2.size):
            j0, j1 = gi[w] * G, min(J, (gi[w] + 1) * G)
            assert 0 <= j0 and j1 <= J
            for j in (j0, j1 - 1) if j1 > j0 else ():
                t3 = (j * n2 + i2[w]) * r0 * r1          # T3 (fwd, adj) and T3b (adj) block
                assert 0 <= t3 and t3 + r0 * r1 <= J * n2 * r0 * r1
                z = (j * n2 + i2[w]) * L                 # Z block (fwd out, adj in)
                assert 0 <= z and z + L <= J * n2 * L
            xt = i2[w] * n0 * n1                         # the plane of the transposed image
            assert xt + n0 * n1 <= N
            if kernel == "adj":
                # gx partials: the workspace holds (J + G_adj - 1) / G_adj planes of N
                gxp = (gi[w] * n2 + i2[w]) * n0 * n1
                assert gxp + n0 * n1 <= ((J + G_adj - 1) // G_adj) * N
