"""Values the paper prints, and what they fix for this build (no GPU)."""
import os

import pytest

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rows():
    out = []
    for line in open(os.path.join(HERE, "paper_grid_counts.txt")):
        if line.strip() and not line.startswith("#"):
            name, nx, ny, nz, total, where = [f.strip() for f in line.split(",", 5)]
            out.append((name, int(nx), int(ny), int(nz), int(total), where))
    return out


def test_verification_mesh_count_includes_one_ghost_layer():
    # Sec. 3 gives 137,924 cells for the 27 x 162 x 27 verification mesh: that total is
    # (27+2)(162+2)(27+2), i.e. the mesh carries one ghost layer around the interior.  Reading taken: neighbours outside the interior grid contribute nothing.
    name, nx, ny, nz, total, _ = [r for r in rows() if r[0] == "verification_bed"][0]
    assert nx * ny * nz != total
    assert (nx + 2) * (ny + 2) * (nz + 2) == total


def test_pic_benchmark_grid_matches_domain_aspect():
    # Sec. 4.1: 10,125,000 cells on a 12 x 12 x 36 cm domain = 150 x 150 x 450 cubic cells
    name, nx, ny, nz, total, _ = [r for r in rows() if r[0] == "pic_strong_scaling"][0]
    assert nx * ny * nz == total
    assert nx / 12 == ny / 12 == nz / 36


def test_benchmark_workloads_are_tall_like_the_papers_beds():
    from paper_2211_15605_amd import workloads as W
    for cfg in (1, 2, 4):
        for g in W.CONFIGS[cfg]["grids"]:
            assert g.ny >= 2 * max(g.nx, g.nz)
