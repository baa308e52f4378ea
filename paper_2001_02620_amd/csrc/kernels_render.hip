// render kernels
