"""MI355X population-dynamics (cloning) sampler for SSEP large deviations."""
