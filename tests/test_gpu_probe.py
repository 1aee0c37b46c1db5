"""The L1 calibration kernel (the benchmark's own library) runs and keeps its loads:
every lane sums the same all-ones words."""
import pytest

pytestmark = pytest.mark.gpu


def test_probe_l1_sums():
    import torch
    from bench import probe_l1
    dev = torch.device("cuda:0")
    buf = torch.ones(1 << 16, dtype=torch.uint8, device=dev)
    blocks, iters = 8, 6
    for mode, units, ub in (("random", 128, 128), ("8_lanes", 64, 64), ("one_line", 16, 16), ("chain", 128, 16)):
        out = torch.full((blocks * 256, 4), -1, dtype=torch.int32, device=dev)
        probe_l1(buf, mode, ub, units, blocks, iters, out)
        torch.cuda.synchronize()
        o = out.cpu().numpy().astype("int64") & 0xFFFFFFFF
        # x and z accumulate by addition, y and w by xor (an even count cancels)
        assert (o[:, 0] == iters * 0x01010101).all() and (o[:, 2] == iters * 0x01010101).all(), mode
        assert (o[:, 1] == 0).all() and (o[:, 3] == 0).all(), mode
