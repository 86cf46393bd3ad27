"""Calibration for the HBM traffic counters: a plain device-to-device copy of
a known size (256 MiB read + 256 MiB written), profiled with the same
FETCH_SIZE / WRITE_SIZE counters as the multiply.  The ratio of counted to
moved bytes is the scale factor applied to the multiply's counters."""
import torch

n = 256 << 20
a = torch.ones(n // 8, dtype=torch.float64, device="cuda")
b = torch.empty_like(a)
for _ in range(3):
    b.copy_(a)
torch.cuda.synchronize()
print("copied", 3 * n, "bytes in 3 launches")
