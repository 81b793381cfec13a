"""Runs the cost-model MLP's forward and gradient kernels three times each on
16384 seeded random samples: the workload of the MFMA counter pass kept in
the profiles (``rocprofv3 --pmc ... -- python3 -m paper_1510_06585_amd.mlp_probe``)."""
import torch

from . import skel as sk


def main(n: int = 16384, reps: int = 3) -> None:
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    P = sk.mlp_param_count()
    params = (torch.rand(P, device="cuda", generator=g) - 0.5) * 0.2
    X = torch.rand(n, 24, device="cuda", generator=g)
    t = torch.rand(n, device="cuda", generator=g)
    y = torch.empty(n, device="cuda")
    grad = torch.empty(P, device="cuda")
    loss = torch.empty(1, device="cuda")
    for _ in range(reps):
        sk.mlp_forward(params, X, y)
        sk.mlp_grad(params, X, t, grad, loss)
    torch.cuda.synchronize()
    print("mlp probe done", flush=True)


if __name__ == "__main__":
    main()
