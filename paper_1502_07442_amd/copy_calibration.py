"""Device copy of a known size, run under rocprofv3 --pmc FETCH_SIZE or
WRITE_SIZE to find how the counters scale to bytes on this GPU: 3 copies of
2^27 float64 (1 GiB each)."""
import torch

n = 1 << 27
x = torch.ones(n, dtype=torch.float64, device="cuda")
y = torch.empty_like(x)
torch.cuda.synchronize()
for _ in range(3):
    y.copy_(x)
torch.cuda.synchronize()
print("copied 3 x 1 GiB", flush=True)
