"""Copy of a known size, run under the HBM traffic counters to calibrate them.

Copies 2 GiB (int64) on the device once; the FETCH_SIZE and WRITE_SIZE
counters of that dispatch divided by 2 GiB give the factor that converts the
counters into bytes.
"""
import torch

N = 1 << 28   # int64 elements = 2 GiB
a = torch.ones(N, dtype=torch.int64, device="cuda")
b = torch.empty_like(a)
torch.cuda.synchronize()
b.copy_(a)
torch.cuda.synchronize()
print(f"copied {N * 8} bytes", flush=True)
