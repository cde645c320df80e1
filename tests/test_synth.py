"""Seeded input generator: reproducibility, layout and the shapes of the
synthetic workloads."""
import numpy as np

import synth

# Known-answer vectors of Philox-4x32-10 published with the Random123 library
# (Salmon et al., SC'11): (counter, key) -> output.
KAT = [
    ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
    ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
    ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
     [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
]


def test_philox_known_answers():
    for ctr, key, out in KAT:
        assert synth.philox(ctr, key) == out


def test_streams_reproducible_and_distributed():
    a = synth.normal(11, 2, 200000)
    assert np.array_equal(a, synth.normal(11, 2, 200000))
    assert np.array_equal(a[1000:1010], synth.normal(11, 2, 10, start=1000))
    assert abs(a.mean()) < 0.01 and abs(a.std() - 1) < 0.01
    u = synth.uniform(11, 1, 200000)
    assert u.min() >= 0 and u.max() < 1 and abs(u.mean() - 0.5) < 0.01


def test_B_blocks_and_columns():
    R = synth.positions_c1()
    B = synth.B_full(1, R, 256, ldB=2080 + 13)
    assert np.all(B[:, 2080:] == 0)
    assert np.array_equal(B[37:50], synth.B_rows(1, R, 37, 13, ldB=2093))
    cols = np.array([0, 5, 2079, 1000])
    assert np.array_equal(synth.B_cols(1, R, 256, cols), B[:, cols])
    # decay envelope: |B| <= a_P * exp(-r^2/2) * |z|; far pairs are tiny
    p_far = synth.pair_index(0, 63)  # corners of the 4x4x4 lattice, r^2 = 3*4.5^2
    assert np.abs(B[:, p_far]).max() < 1e-10


def test_lattices():
    assert synth.positions_c1().shape == (64, 3)
    R2 = synth.positions_c2()
    assert R2.shape == (1024, 3)
    assert np.array_equal(R2[0], R2[2]) and not np.array_equal(R2[2], R2[3])
    assert synth.positions_c3().shape == (2048, 3)
    R5 = synth.positions_c5(3)
    assert R5.shape == (128, 3) and np.abs(R5 - synth.lattice(8, 4, 4)).max() < 1.0
    sizes = synth.batch_sizes()
    assert sizes.size == 256 and sizes.min() >= 40 and sizes.max() <= 400
    Rc = synth.cluster_positions(4001, 137)
    assert Rc.shape == (137, 3) and len({tuple(r) for r in Rc}) == 137
    # connected: every site has a lattice neighbour in the cluster
    d = np.linalg.norm(Rc[:, None] - Rc[None], axis=-1)
    assert np.all(np.sort(d, 1)[:, 1] < synth.SPACING + 1e-9)


def test_occupied_orbitals():
    C = synth.C_occ(1, 64, 16)
    assert np.allclose(C.T @ C, np.eye(16), atol=1e-13)
    D = 2 * C @ C.T
    assert np.allclose(D @ D, 2 * D, atol=1e-12)
    assert abs(np.trace(D) - 32) < 1e-12


def test_core_hamiltonian():
    R = synth.positions_c5(5)
    H = synth.core_hamiltonian(5, R)
    assert np.array_equal(H, H.T)
    d = np.diag(H)
    assert d.min() > -5.5 and d.max() < -0.5
