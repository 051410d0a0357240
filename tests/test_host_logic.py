"""Host-side logic of the binding and the library's size functions (no GPU:
the checks run before any device call)."""
import numpy as np
import pytest
import torch

from paper_2212_10550_amd import lib as K


def test_occ_words_is_whole_bricks():
    for G in (1, 7, 8, 16, 37, 128, 2048):
        nb, nbz = -(-G // 8), -(-G // 16)
        assert K.occ_words(G) == nb * nb * nbz * 32
    assert K.occ_words(0) == 0 and K.occ_words(2049) == 0
    assert K.occ_words(128) == (128 ** 3) // 32  # no padding at multiples of 16


def test_march_workspace_covers_masks_and_scan():
    for R, steps in ((1, 1), (8192, 128), (291600, 128), (1166400, 128), (1000, 300), (65535, 128), (65536, 128)):
        nblk = -(-R // (16 if R >= 65536 else 4))  # rays per workgroup: 4 per wave from 65536 rays, else 1
        need = 8 * nblk + 8 * (-(-nblk // 4096)) + 8 * R * (-(-steps // 64)) + 4 * R
        assert K.march_workspace_size(R, steps) >= need
    assert K.march_workspace_size(-1, 128) == 0 and K.march_workspace_size(10, -1) == 0


def test_backward_and_regulariser_workspaces():
    assert K.hashgrid_encode_bwd_workspace_size(36503, 16) >= 4 * 3 * 16 * 36503
    assert K.hashgrid_encode_bwd_workspace_size(-1, 16) == 0
    # binned table gradient: 12-byte records, 8 per sample and level, dominate
    n = K.hashgrid_table_grad_workspace_size(36503, 16, 1 << 19)
    assert 12 * 8 * 16 * 36503 <= n < 12 * 8 * 16 * 36503 + (8 << 20)
    assert K.hashgrid_table_grad_workspace_size(36503, 16, 1 << 22) > 0  # 16384 tiles of 4096 entries
    assert K.hashgrid_table_grad_workspace_size(36503, 16, 1 << 23) == 0  # beyond the tile limit
    assert K.hashgrid_table_grad_workspace_size(1 << 26, 16, 1 << 19) == 0  # 8 L S >= 2^32 records
    with pytest.raises(ValueError):
        K.hashgrid_table_grad_workspace_size(100, 16, 3 << 18)
    assert K.density_reg_workspace_size(10 ** 6) >= 4 * min(-(-10 ** 6 // 256), 1024)
    assert K.occgrid_build_workspace_size(64, 16, 2, K.F32, 64, 64, 32) >= 64 ** 3 * (12 + 12 + 4 + 12 + 2 + 128)
    assert K.occgrid_build_workspace_size(257, 16, 2, K.F32, 64, 64, 32) == 0
    assert K.occgrid_build_workspace_size(64, 16, 2, K.BF16, 64, 64, 32) < \
        K.occgrid_build_workspace_size(64, 16, 2, K.F32, 64, 64, 32)


def test_binding_rejects_bad_shapes_before_any_device_call():
    cpu = torch.zeros
    with pytest.raises(ValueError):
        K.occ_pack(cpu(4, 4, 5, dtype=torch.uint8), cpu(64, dtype=torch.int32))
    with pytest.raises(ValueError):
        K.occ_pack(cpu(16, 16, 16, dtype=torch.uint8), cpu(10, dtype=torch.int32))
    with pytest.raises(ValueError):
        K.adam(cpu(10), cpu(9), cpu(10), cpu(10), 1e-2)
    with pytest.raises(ValueError):
        K.occ_from_density(cpu(100), 8, 0.5, 1, cpu(K.occ_words(8), dtype=torch.int32))
    # shapes fine, but host tensors: refused by the pointer check
    with pytest.raises(TypeError):
        K.adam(cpu(10), cpu(10), cpu(10), cpu(10), 1e-2)


def test_flags_are_distinct_bits():
    flags = [K.OVERWRITE, K.TABLE_COARSE, K.TABLE_FINE]
    assert all(f & (f - 1) == 0 for f in flags) and len(set(flags)) == 3


def test_autograd_front_end_dtype_checks():
    from paper_2212_10550_amd import autograd as A
    cfg = A.HashConfig(16.0, 1.38, (0, 0, 0, 1, 1, 1))
    with pytest.raises(TypeError):
        A.hash_encode(torch.zeros(3, 4), torch.zeros(4, dtype=torch.int16), torch.zeros(16, 64, 2).half(), cfg)
    with pytest.raises(TypeError):
        A.mlp(torch.zeros(16, 4, 2).bfloat16(), torch.zeros(4, dtype=torch.int16), torch.zeros(6532))
