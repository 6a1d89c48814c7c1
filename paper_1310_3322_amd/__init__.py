"""MI355X-native discrete-HMM bank: forward log-likelihoods, recognition and the
Baum-Welch E-step gradient on gfx950 (HIP kernels behind include/hmm.h).

The HIP library is loaded on first use by paper_1310_3322_amd.hmm; importing the
package itself needs neither the library nor a GPU.
"""
__all__ = ["hmm", "workloads"]
