"""One device-to-device copy of 2^28 float32 (1 GiB): the reference kernel for
scaling the HBM byte counters (FETCH_SIZE, WRITE_SIZE) of rocprofv3."""
import torch

a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
b = torch.empty_like(a)
torch.cuda.synchronize()
b.copy_(a)
torch.cuda.synchronize()
print("copied", a.numel() * 4, "bytes")
