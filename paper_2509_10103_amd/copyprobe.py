"""Calibration workload for hardware byte counters: one plain device-to-device
copy of 1 GiB (its FETCH_SIZE / WRITE_SIZE per dispatch should read 1 GiB)."""
import torch

if __name__ == "__main__":
    a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print("copied", b.numel(), "bytes")
